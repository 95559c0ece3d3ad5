// The ANOVA kernel matrix-vector product y = sum_l eta_l K_l x (Section 3),
// every window by NFFT fast summation:
//   spread   g = sum_i x_i phi(. - x_i)           (adjoint NFFT, inner sum)
//   convolve h = (T_x (x) T_y (x) T_z) g          (FFT, times B, inverse FFT)
//   gather   f_j = sum_cells h phi(x_j - .)       (forward NFFT, outer sum)
//   sum      y_j = sum_l eta_l f_j^{(l)}          (fixed window order, FP64)
//
// Work decomposition (gfx950, wave64). Points of a window are sorted by
// (column (cx, cy), layer cz) of their base cell. A work item is a run of
// consecutive sorted points of one column. For 3-feature windows a wavefront
// takes 64/W work items (W = 2m taps per axis), one per group of W lanes: lane
// (group, a) owns the x-tap a of its item's footprint and keeps the W x W block
// (y-tap b, z-cell c) of grid values in registers, so each point's weights are
// needed by only W lanes (staged in LDS once per round of W points). As the run
// advances in z, finished z-cells are written (spread) or new ones loaded
// (gather). 1- and 2-feature windows use one lane per work item. No atomics
// anywhere: each work item writes its own slab of partial sums and the fold
// kernel adds the slabs that cover a cell in a fixed order, so results are
// reproducible bit for bit.
#include <cstring>
#include <mutex>
#include <string>

#include "plan.hpp"

namespace anv {

namespace {

constexpr int kThreads = 256;
inline unsigned nblocks(int64_t n, int t = kThreads) { return unsigned((n + t - 1) / t); }

// Asynchronous staging of point records straight into LDS (gfx950 LDS DMA,
// 16 bytes per lane per instruction). The chunk region holds CH records of RS
// elements (REC data + padding); each 1 KB instruction slot maps to a record
// element, padding slots and points past the item read a valid dummy record.
template <class WT, int REC, int RS, int CH>
__device__ inline void stage_records_async(WT* lds, const WT* __restrict__ wts, int64_t base, int cstart,
                                           int count, int lane) {
    constexpr int RB = RS * int(sizeof(WT));
    constexpr int BYTES = CH * RB;
    static_assert(BYTES % 1024 == 0, "chunk region must be whole 1 KB DMA slots");
    static_assert(RB % 16 == 0 && (REC * int(sizeof(WT))) % 16 == 0, "records must be 16-byte pieces");
#pragma unroll
    for (int j = 0; j < BYTES / 1024; ++j) {
        const int o = j * 1024 + lane * 16;
        const int pnt = o / RB;
        const int e = (o % RB) / int(sizeof(WT));
        const int pt = cstart + pnt;
        const bool valid = e < REC && pt < count;
        const WT* src = valid ? wts + (base + pt) * REC + e : wts + base * REC;
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                         (__attribute__((address_space(3))) void*)(lds + j * (1024 / int(sizeof(WT)))),
                                         16, 0, 0);
    }
}

// 64 input values (doubles) of points cstart .. cstart+63 into a 1 KB LDS slot
// (lanes 0..31 move two values each; the input array carries two padding entries)
__device__ inline void stage_values_async(double* lds, const double* __restrict__ vs, int64_t base, int cstart,
                                          int count, int lane) {
    const int pt = cstart + 2 * lane;
    const bool valid = lane < 32 && pt < count;
    const double* src = valid ? vs + base + pt : vs + base;
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                     (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}

__device__ inline void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

// Layer starts of a 3-feature work item (its points of layer z0 + i are
// [ls[i], ls[i + 1])), held one entry per lane (an item spans at most
// kItemLayers layers, so its z1 - z0 + 2 entries fit) and read with readlane:
// the layer index is the same in every lane, so the layer loop issues no
// memory access for them.
struct LayerStarts {
    int v;
    __device__ LayerStarts(const int32_t* __restrict__ ls, int count, int lane) { v = lane < count ? ls[lane] : 0; }
    __device__ void get(int i, int& p, int& q) const {
        p = __builtin_amdgcn_readlane(v, i);
        q = __builtin_amdgcn_readlane(v, i + 1);
    }
};

// LDS reads of staged point data for 8 taps per axis. They are written as asm
// with the wait for their own completion inside the block: the compiler would
// otherwise make every LDS read wait for all DMA in flight, the prefetch of the
// next chunk included. Staged data are read only after the explicit wait at the
// chunk switch.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ inline uint32_t lds_addr(const void* p) { return static_cast<uint32_t>(reinterpret_cast<uintptr_t>(p)); }

// one tap's x weight (at xa), an input value (at va) and the 8 y and 8 z
// weights (16 consecutive elements at yz, 16-byte aligned)
__device__ inline void lds_point8(uint32_t xa, uint32_t va, uint32_t yz, double& wx, double& v, double (&wy)[8],
                                  double (&wz)[8]) {
    d2v q[8];
    asm volatile(
        "ds_read_b64 %0, %10\n\t"
        "ds_read_b64 %1, %11\n\t"
        "ds_read_b128 %2, %12\n\t"
        "ds_read_b128 %3, %12 offset:16\n\t"
        "ds_read_b128 %4, %12 offset:32\n\t"
        "ds_read_b128 %5, %12 offset:48\n\t"
        "ds_read_b128 %6, %12 offset:64\n\t"
        "ds_read_b128 %7, %12 offset:80\n\t"
        "ds_read_b128 %8, %12 offset:96\n\t"
        "ds_read_b128 %9, %12 offset:112\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(wx), "=&v"(v), "=&v"(q[0]), "=&v"(q[1]), "=&v"(q[2]), "=&v"(q[3]), "=&v"(q[4]), "=&v"(q[5]),
          "=&v"(q[6]), "=&v"(q[7])
        : "v"(xa), "v"(va), "v"(yz)
        : "memory");
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        wy[2 * i] = q[i].x;
        wy[2 * i + 1] = q[i].y;
        wz[2 * i] = q[4 + i].x;
        wz[2 * i + 1] = q[4 + i].y;
    }
}

__device__ inline void lds_point8(uint32_t xa, uint32_t va, uint32_t yz, float& wx, double& v, float (&wy)[8],
                                  float (&wz)[8]) {
    f4v q[4];
    asm volatile(
        "ds_read_b32 %0, %6\n\t"
        "ds_read_b64 %1, %7\n\t"
        "ds_read_b128 %2, %8\n\t"
        "ds_read_b128 %3, %8 offset:16\n\t"
        "ds_read_b128 %4, %8 offset:32\n\t"
        "ds_read_b128 %5, %8 offset:48\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(wx), "=&v"(v), "=&v"(q[0]), "=&v"(q[1]), "=&v"(q[2]), "=&v"(q[3])
        : "v"(xa), "v"(va), "v"(yz)
        : "memory");
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            wy[4 * i + j] = q[i][j];
            wz[4 * i + j] = q[2 + i][j];
        }
}

// Per-layer sums over the 8 lane groups of the 3-feature spread (8 taps, row
// stride 72 elements): lane l writes its 8 values (y taps b) at red[b * 72 + l]
// and reads the 8 group values of its own (a, b) at red[b * 72 + g * 8 + a],
// g = 0..7. The block is one wavefront, whose LDS instructions run in order, so
// no barrier is needed between the writes and the reads.
__device__ inline void lds_red8(uint32_t wa, uint32_t ra, const double (&w)[8], double (&r)[8]) {
    asm volatile(
        "ds_write_b64 %0, %1\n\t"
        "ds_write_b64 %0, %2 offset:576\n\t"
        "ds_write_b64 %0, %3 offset:1152\n\t"
        "ds_write_b64 %0, %4 offset:1728\n\t"
        "ds_write_b64 %0, %5 offset:2304\n\t"
        "ds_write_b64 %0, %6 offset:2880\n\t"
        "ds_write_b64 %0, %7 offset:3456\n\t"
        "ds_write_b64 %0, %8 offset:4032"
        :
        : "v"(wa), "v"(w[0]), "v"(w[1]), "v"(w[2]), "v"(w[3]), "v"(w[4]), "v"(w[5]), "v"(w[6]), "v"(w[7])
        : "memory");
    asm volatile(
        "ds_read_b64 %0, %8\n\t"
        "ds_read_b64 %1, %8 offset:64\n\t"
        "ds_read_b64 %2, %8 offset:128\n\t"
        "ds_read_b64 %3, %8 offset:192\n\t"
        "ds_read_b64 %4, %8 offset:256\n\t"
        "ds_read_b64 %5, %8 offset:320\n\t"
        "ds_read_b64 %6, %8 offset:384\n\t"
        "ds_read_b64 %7, %8 offset:448\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]), "=&v"(r[7])
        : "v"(ra)
        : "memory");
}

__device__ inline void lds_red8(uint32_t wa, uint32_t ra, const float (&w)[8], float (&r)[8]) {
    asm volatile(
        "ds_write_b32 %0, %1\n\t"
        "ds_write_b32 %0, %2 offset:288\n\t"
        "ds_write_b32 %0, %3 offset:576\n\t"
        "ds_write_b32 %0, %4 offset:864\n\t"
        "ds_write_b32 %0, %5 offset:1152\n\t"
        "ds_write_b32 %0, %6 offset:1440\n\t"
        "ds_write_b32 %0, %7 offset:1728\n\t"
        "ds_write_b32 %0, %8 offset:2016"
        :
        : "v"(wa), "v"(w[0]), "v"(w[1]), "v"(w[2]), "v"(w[3]), "v"(w[4]), "v"(w[5]), "v"(w[6]), "v"(w[7])
        : "memory");
    asm volatile(
        "ds_read_b32 %0, %8\n\t"
        "ds_read_b32 %1, %8 offset:32\n\t"
        "ds_read_b32 %2, %8 offset:64\n\t"
        "ds_read_b32 %3, %8 offset:96\n\t"
        "ds_read_b32 %4, %8 offset:128\n\t"
        "ds_read_b32 %5, %8 offset:160\n\t"
        "ds_read_b32 %6, %8 offset:192\n\t"
        "ds_read_b32 %7, %8 offset:224\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]), "=&v"(r[7])
        : "v"(ra)
        : "memory");
}

// Block b of a launch belongs to job j with off[j] <= b < off[j + 1]; returns j
// and turns b into the job's local block index.
__device__ inline int job_of(const MvLaunch& L, int& b) {
    int j = 0;
    while (j + 1 < L.njobs && L.off[j + 1] <= b) ++j;
    b -= L.off[j];
    return j;
}

__global__ void k_permute(const MvLaunch ML) {
    int b = blockIdx.x;
    const MvJob& J = ML.job[job_of(ML, b)];
    const int64_t t = b * (int64_t)blockDim.x + threadIdx.x;
    if (t >= J.N * J.P) return;
    J.vs[t] = J.x[J.perm[t]];
}

// 3-feature windows: one work item (a long run of one column) per wavefront.
// The run is swept layer by layer; within a layer its points are dealt to the
// 64/W lane groups, W points... one per group per step. Lane (group, a) keeps
// the W x W block (y-tap b, z-cell c) of its group's partial sums; when a layer
// is complete the groups' values for it are added in group order through LDS
// and the wave writes one slab row [a][b]. Point data are staged in LDS in
// chunks of 64 consecutive points.
template <int W, class WT>
__device__ __forceinline__ void spread_grp(const MvJob& J, const int blk) {
    const Segment* __restrict__ segs = J.segs;
    const int32_t* __restrict__ lstart = J.lstart;
    const int32_t* __restrict__ lstart_off = J.lstart_off;
    const WinDev* __restrict__ wins = J.wins;
    const uint8_t* __restrict__ alone = J.alone;
    const WT* __restrict__ wts = static_cast<const WT*>(J.wts);
    const double* __restrict__ vs = J.vs;
    const int64_t N = J.N;
    WT* __restrict__ slab = static_cast<WT*>(J.slab);
    WT* __restrict__ tgt = static_cast<WT*>(J.ca);
    constexpr int G = 64 / W;                 // lane groups
    constexpr int REC = rec_stride(W, int(sizeof(WT)));
    // staged points and record padding (the padding spreads the groups over the
    // LDS banks); FP64 records of 8 taps per axis are staged 32 at a time, so
    // that the block's LDS (about 21 KB instead of 33 KB) admits more wavefronts
    constexpr bool kHalf = sizeof(WT) == 8 && W == 8;
    constexpr int CH = kHalf ? 32 : 64;
    constexpr int PADR = (kHalf ? 32 : 16) / int(sizeof(WT));
    constexpr int RS = REC + PADR;
    constexpr int STEP = CH - G;               // chunk c holds points [c*STEP, c*STEP + CH)
    __shared__ __align__(16) WT stw[2][CH * RS];
    __shared__ __align__(16) double stv[2][128];
    // per-layer group sums: plane b holds [g][a] (consecutive lanes write consecutive
    // elements); the plane stride 72 = 64 + 8 spreads the (a, b) readers over all banks
    constexpr int RP = 64 + 8;
    __shared__ __align__(16) WT red[W * RP];
    const int sid = J.wave_items[J.wave_off[3] + blk];
    const Segment sg = segs[sid];
    const int lane = threadIdx.x;
    const int g = lane / W, a = lane % W;
    const bool lane_ok = g < G;
    const int64_t base = int64_t(sg.win) * N + sg.start;
    const int32_t* ls = lstart + lstart_off[sid];
    WT acc[W][W];
#pragma unroll
    for (int b = 0; b < W; ++b)
#pragma unroll
        for (int c = 0; c < W; ++c) acc[b][c] = WT(0);
    // an item alone in its column has no overlapping neighbour: its layers go
    // straight to the fold's target-major buffer (target line (cx+a, cy+b),
    // footprint position (a, b)); otherwise to its slab
    const bool direct = alone[sid] != 0;
    WT* out = slab + sg.off;
    WT* tout = tgt;
    int64_t tstride = 1;
    {
        const WinDev& wd = wins[sg.win];
        const int cx = sg.col / wd.nb[1], cy = sg.col % wd.nb[1];
        const int ta = lane / W, tb = lane % W;  // footprint position written by this lane
        tout = tgt + wd.tgt_off + ((int64_t(cx + ta) * wd.E[1] + (cy + tb)) * (W * W) + lane) * wd.E[2] + sg.z0;
        tstride = 1;
    }
    int cc = -1;
    LayerStarts lsw(ls, sg.z1 - sg.z0 + 2, lane);
    stage_records_async<WT, REC, RS, CH>(stw[0], wts, base, 0, sg.count, lane);
    stage_values_async(stv[0], vs, base, 0, sg.count, lane);
    auto flush = [&](int layer, int c) {  // sum acc[.][c] over groups -> row `layer`
        if constexpr (W == 8) {
            WT w8[W], r8[W];
#pragma unroll
            for (int b = 0; b < W; ++b) w8[b] = acc[b][c];
            lds_red8(lds_addr(&red[lane]), lds_addr(&red[(lane % W) * RP + lane / W]), w8, r8);
            WT t = WT(0);
#pragma unroll
            for (int q = 0; q < G; ++q) t += r8[q];
            if (direct)
                tout[int64_t(layer) * tstride] = t;
            else
                out[int64_t(layer) * (W * W) + lane] = t;
            return;
        }
        if (lane_ok) {
#pragma unroll
            for (int b = 0; b < W; ++b) red[b * RP + g * W + a] = acc[b][c];
        }
        __syncthreads();
        if (lane < W * W) {
            const int ra = lane / W, rb = lane % W;
            WT t = WT(0);
#pragma unroll
            for (int q = 0; q < G; ++q) t += red[rb * RP + q * W + ra];
            if (direct)
                tout[int64_t(layer) * tstride] = t;
            else
                out[int64_t(layer) * (W * W) + lane] = t;
        }
        __syncthreads();
    };
    for (int z = sg.z0; z <= sg.z1; ++z) {
        int p, q;
        lsw.get(z - sg.z0, p, q);
        for (int k = p; k < q; k += G) {
            const int c = k / STEP;
            if (c > cc) {  // chunk c has landed; start moving chunk c+1 into the other buffer
                wait_vmem();
                __syncthreads();
                cc = c;
                if ((c + 1) * STEP < sg.count) {
                    stage_records_async<WT, REC, RS, CH>(stw[(c + 1) & 1], wts, base, (c + 1) * STEP, sg.count, lane);
                    stage_values_async(stv[(c + 1) & 1], vs, base, (c + 1) * STEP, sg.count, lane);
                }
            }
            const int cbase = c * STEP;
            const int pt = k + g;
            if (lane_ok && pt < q) {
                const WT* w = &stw[c & 1][(pt - cbase) * RS];
                if constexpr (W == 8) {
                    WT wx, wy[W], wz[W];
                    double v;
                    lds_point8(lds_addr(w + a), lds_addr(&stv[c & 1][pt - cbase]), lds_addr(w + W), wx, v, wy, wz);
                    const WT vx = WT(v) * wx;
#pragma unroll
                    for (int b = 0; b < W; ++b) {
                        const WT cb = vx * wy[b];
#pragma unroll
                        for (int c = 0; c < W; ++c) acc[b][c] += cb * wz[c];
                    }
                } else {
                    const WT vx = WT(stv[c & 1][pt - cbase]) * w[a];
                    WT wz[W];
#pragma unroll
                    for (int c = 0; c < W; ++c) wz[c] = w[2 * W + c];
#pragma unroll
                    for (int b = 0; b < W; ++b) {
                        const WT cb = vx * w[W + b];
#pragma unroll
                        for (int c = 0; c < W; ++c) acc[b][c] += cb * wz[c];
                    }
                }
            }
        }
        flush(z - sg.z0, 0);
#pragma unroll
        for (int b = 0; b < W; ++b) {
#pragma unroll
            for (int c = 0; c < W - 1; ++c) acc[b][c] = acc[b][c + 1];
            acc[b][W - 1] = WT(0);
        }
    }
#pragma unroll
    for (int c = 0; c < W - 1; ++c) flush(sg.z1 + 1 + c - sg.z0, c);
}

// 1- and 2-feature windows: one lane per work item; WY = W for two features
// (y taps in registers), 1 for one feature. Slab layout [layer][b].
template <int W, int WY, class WT>
__device__ __forceinline__ void spread_lane(const MvJob& J, const int blk) {
    const Segment* __restrict__ segs = J.segs;
    const int32_t* __restrict__ zq = J.zq;
    const WT* __restrict__ wts = static_cast<const WT*>(J.wts);
    const double* __restrict__ vs = J.vs;
    const int64_t N = J.N;
    WT* __restrict__ slab = static_cast<WT*>(J.slab);
    const int sid = J.wave_items[J.wave_off[WY == 1 ? 1 : 2] + blk * 64 + threadIdx.x];
    if (sid < 0) return;
    const Segment sg = segs[sid];
    const int64_t base = int64_t(sg.win) * N + sg.start;
    WT acc[WY][W];
#pragma unroll
    for (int b = 0; b < WY; ++b)
#pragma unroll
        for (int c = 0; c < W; ++c) acc[b][c] = WT(0);
    int zr = sg.z0;
    WT* out = slab + sg.off;
    for (int k = 0; k < sg.count; ++k) {
        const int64_t gi = base + k;
        const int zj = zq[gi];
        while (zr < zj) {
#pragma unroll
            for (int b = 0; b < WY; ++b) out[int64_t(zr - sg.z0) * WY + b] = acc[b][0];
#pragma unroll
            for (int b = 0; b < WY; ++b) {
#pragma unroll
                for (int c = 0; c < W - 1; ++c) acc[b][c] = acc[b][c + 1];
                acc[b][W - 1] = WT(0);
            }
            ++zr;
        }
        const WT* w = wts + gi * rec_stride(W, int(sizeof(WT)));
        const WT v = WT(vs[gi]);
        WT wz[W];
#pragma unroll
        for (int c = 0; c < W; ++c) wz[c] = w[2 * W + c];
#pragma unroll
        for (int b = 0; b < WY; ++b) {
            const WT cb = v * w[W + b];
#pragma unroll
            for (int c = 0; c < W; ++c) acc[b][c] += cb * wz[c];
        }
    }
#pragma unroll
    for (int c = 0; c < W; ++c)
#pragma unroll
        for (int b = 0; b < WY; ++b) out[int64_t(zr - sg.z0 + c) * WY + b] = acc[b][c];
}

// Spreading of every window of the launch's plans in one launch: the grouped
// work items of 3-feature windows first (longest first), then the one-lane
// items of 2- and 1-feature windows, which fill the machine while the last
// long items finish.
template <int W, class WT>
__global__ __launch_bounds__(64) void k_spread(const MvLaunch ML) {
    int blk = blockIdx.x;
    const MvJob& J = ML.job[job_of(ML, blk)];
    if (blk < J.nwave[3])
        spread_grp<W, WT>(J, blk);
    else if (blk < J.nwave[3] + J.nwave[2])
        spread_lane<W, W, WT>(J, blk - J.nwave[3]);
    else
        spread_lane<W, 1, WT>(J, blk - J.nwave[3] - J.nwave[2]);
}

// Fold, step A for 3-feature windows: one wavefront per (window, column, layer). Lane (a, b) adds, in
// item order, the slab values that the column's work items wrote for layer L
// at footprint position (a, b), and stores the sum under its TARGET line
// (cx + a, cy + b): tgt[window][target x][target y][a, b][layer]. Every
// (target, (a, b)) has exactly one source column, so no two lanes write the
// same element.
template <class WT>
__global__ __launch_bounds__(256) void k_fold_cols(const MvLaunch ML) {
    int blk = blockIdx.x;
    const MvJob& J = ML.job[job_of(ML, blk)];
    const WinDev* __restrict__ wins = J.wins;
    const int32_t P = J.P;
    const int64_t nlist = J.nflist3;  // entries of 3-feature windows
    const int64_t* __restrict__ flist = J.flist;
    const int2* __restrict__ fold = J.fold;
    const int64_t* __restrict__ sbase = J.sbase;
    const WT* __restrict__ slab = static_cast<const WT*>(J.slab);
    WT* __restrict__ tgt = static_cast<WT*>(J.ca);
    const int64_t fi = int64_t(blk) * 4 + threadIdx.x / 64;
    if (fi >= nlist) return;
    const int64_t f = flist[fi];
    int l = 0;
    while (l + 1 < P && wins[l + 1].fold_off <= f) ++l;
    const WinDev& wd = wins[l];
    const int lane = threadIdx.x % 64;
    const int64_t fl = f - wd.fold_off;
    const int L = int(fl % wd.E[2]);
    const int64_t col = fl / wd.E[2];
    const int cx = int(col / wd.nb[1]), cy = int(col % wd.nb[1]);
    // lane = (part, footprint position): the items covering the cell are dealt
    // to the parts in turn (windows with fewer than 64 positions use the spare
    // lanes), and the parts' sums are added in part order
    const int lanes = wd.lanes, parts = 64 / lanes;
    const int pos = lane % lanes, part = lane / lanes;
    const int a = pos / wd.Wslot[1], b = pos % wd.Wslot[1];
    const int2 r = fold[f];
    double acc = 0.0;
    if (part < parts) {
        const int64_t row = int64_t(L) * lanes + pos;
        int s = r.x + part;
        for (; s + 3 * parts < r.y; s += 4 * parts) {
            const int64_t o0 = sbase[s], o1 = sbase[s + parts], o2 = sbase[s + 2 * parts], o3 = sbase[s + 3 * parts];
            const WT v0 = slab[o0 + row], v1 = slab[o1 + row], v2 = slab[o2 + row], v3 = slab[o3 + row];
            acc += double(v0);
            acc += double(v1);
            acc += double(v2);
            acc += double(v3);
        }
        for (; s < r.y; s += parts) acc += double(slab[sbase[s] + row]);
    }
    double tot = 0.0;
    for (int q = 0; q < parts; ++q) tot += __shfl(acc, q * lanes + pos, 64);
    acc = tot;
    if (lane >= wd.lanes) return;
    const int64_t t = ((int64_t(cx + a) * wd.E[1] + (cy + b)) * wd.lanes + pos) * wd.E[2] + L;
    tgt[wd.tgt_off + t] = WT(acc);
}

// Fold, step A for 1- and 2-feature windows. Their work items are short (one
// lane each), so a cell gathers hundreds of them: one block per (window,
// column, layer), thread = (part, footprint position) with 256 / lanes parts
// taking the items in turn; the parts' sums are added in part order.
template <class WT>
__global__ __launch_bounds__(256) void k_fold_cols_wide(const MvLaunch ML) {
    int blk = blockIdx.x;
    const MvJob& J = ML.job[job_of(ML, blk)];
    const int64_t fi = J.nflist3 + blk;
    if (fi >= J.nflist) return;
    const WinDev* __restrict__ wins = J.wins;
    const int64_t* __restrict__ sbase = J.sbase;
    const WT* __restrict__ slab = static_cast<const WT*>(J.slab);
    WT* __restrict__ tgt = static_cast<WT*>(J.ca);
    const int64_t f = J.flist[fi];
    int l = 0;
    while (l + 1 < J.P && wins[l + 1].fold_off <= f) ++l;
    const WinDev& wd = wins[l];
    const int lanes = wd.lanes, parts = 256 / lanes;
    const int t = threadIdx.x, pos = t % lanes, part = t / lanes;
    const int64_t fl = f - wd.fold_off;
    const int L = int(fl % wd.E[2]);
    const int2 r = J.fold[f];
    double acc = 0.0;
    if (part < parts) {
        const int64_t row = int64_t(L) * lanes + pos;
        int s = r.x + part;
        for (; s + 3 * parts < r.y; s += 4 * parts) {
            const int64_t o0 = sbase[s], o1 = sbase[s + parts], o2 = sbase[s + 2 * parts], o3 = sbase[s + 3 * parts];
            const WT v0 = slab[o0 + row], v1 = slab[o1 + row], v2 = slab[o2 + row], v3 = slab[o3 + row];
            acc += double(v0);
            acc += double(v1);
            acc += double(v2);
            acc += double(v3);
        }
        for (; s < r.y; s += parts) acc += double(slab[sbase[s] + row]);
    }
    __shared__ double red[256];
    red[t] = acc;
    __syncthreads();
    if (t >= lanes) return;
    double tot = 0.0;
    for (int q = 0; q < parts; ++q) tot += red[q * lanes + pos];
    const int64_t col = fl / wd.E[2];
    const int cx = int(col / wd.nb[1]), cy = int(col % wd.nb[1]);
    const int a = pos / wd.Wslot[1], b = pos % wd.Wslot[1];
    const int64_t tt = ((int64_t(cx + a) * wd.E[1] + (cy + b)) * lanes + pos) * wd.E[2] + L;
    tgt[wd.tgt_off + tt] = WT(tot);
}

// Fold step B fused with the y and z passes of the grid convolution. One block
// per (x slice, window): each cell of the slice adds the footprint positions of
// its target line in (a, b) order (only source columns that exist and whose
// layer range covers the cell contribute), then T_y and T_z are applied in LDS
// and the slice is written as g1[x][y][z].
// FP64: blocks of 512 threads, whose 256 registers per lane hold the fold's loads
// without spilling (1024-thread blocks have 128)
template <class WT>
constexpr int fold_conv1_threads() { return sizeof(WT) == 8 ? 512 : 1024; }
template <int W, class WT>
__global__ __launch_bounds__(fold_conv1_threads<WT>()) void k_fold_conv_yz(const MvLaunch ML) {
    extern __shared__ double sm[];
    int blk = blockIdx.x;
    const MvJob& J = ML.job[job_of(ML, blk)];
    const double* __restrict__ tmat = J.tmat;
    const int2* __restrict__ crange = J.crange;
    const WT* __restrict__ tgt = static_cast<const WT*>(J.ca);
    WT* __restrict__ g1 = static_cast<WT*>(J.g);
    const int l = blk / J.emax[0];
    const WinDev& wd = J.wins[l];
    const int x = blk % J.emax[0];
    if (x >= wd.E[0]) return;
    const int Ey = wd.E[1], Ez = wd.E[2];
    const int S = Ey * Ez;
    double* s0 = sm;           // slice [y][z]
    double* s1 = sm + S;       // after the y pass
    double* ty = s1 + S;       // T_y
    double* tz = ty + Ey * Ey; // T_z
    for (int e = threadIdx.x; e < Ey * Ey; e += blockDim.x) ty[e] = tmat[wd.t_off[1] + e];
    for (int e = threadIdx.x; e < Ez * Ez; e += blockDim.x) tz[e] = tmat[wd.t_off[2] + e];
    const int wx = wd.Wslot[0], wy = wd.Wslot[1];
    // layer ranges of the source columns this slice can see: cx in [x-W+1, x]
    __shared__ int2 rng[W][64 + 1];
    const int nby = wd.nb[1];
    for (int e = threadIdx.x; e < W * nby; e += blockDim.x) {
        const int a = e / nby, cy = e % nby, cx = x - a;
        rng[a][cy] = (a < wx && cx >= 0 && cx < wd.nb[0]) ? crange[wd.col_off + int64_t(cx) * nby + cy]
                                                          : make_int2(1, 0);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < S; e += blockDim.x) {
        const int y = e / Ez, z = e % Ez;
        const WT* tl = tgt + wd.tgt_off + (int64_t(x) * Ey + y) * wd.lanes * Ez + z;
        WT v[W][W];
        bool ok[W][W];
#pragma unroll
        for (int a = 0; a < W; ++a)
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const int cy = y - b;
                const int2 rr = (b < wy && cy >= 0 && cy < nby) ? rng[a][cy] : make_int2(1, 0);
                ok[a][b] = z >= rr.x && z <= rr.y;
                v[a][b] = tl[ok[a][b] ? int64_t(a * wy + b) * Ez : 0];
            }
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < W; ++a)
#pragma unroll
            for (int b = 0; b < W; ++b) acc += ok[a][b] ? double(v[a][b]) : 0.0;
        s0[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < S; e += blockDim.x) {  // y pass
        const int y = e / Ez, z = e % Ez;
        double acc = 0.0;
        for (int k = 0; k < Ey; ++k) acc += ty[y * Ey + k] * s0[k * Ez + z];
        s1[e] = acc;
    }
    __syncthreads();
    WT* out = g1 + wd.grid_off + int64_t(x) * S;
    for (int e = threadIdx.x; e < S; e += blockDim.x) {  // z pass
        const int y = e / Ez, z = e % Ez;
        double acc = 0.0;
        // T_z is symmetric (entries depend on |i - k|): read it by column, so
        // that consecutive lanes (consecutive z) hit consecutive LDS banks
        for (int k = 0; k < Ez; ++k) acc += tz[k * Ez + z] * s1[y * Ez + k];
        out[e] = WT(acc);
    }
}

// x pass of the grid convolution, one block per (y slice, window); the result
// is stored as h[x][z][y], the layout the gather reads.
template <class WT>
__global__ __launch_bounds__(256) void k_conv_x(const MvLaunch ML) {
    extern __shared__ double sm[];
    int blk = blockIdx.x;
    const MvJob& J = ML.job[job_of(ML, blk)];
    const double* __restrict__ tmat = J.tmat;
    const WT* __restrict__ g1 = static_cast<const WT*>(J.g);
    WT* __restrict__ h = static_cast<WT*>(J.h);
    const int l = blk / J.emax[1];
    const WinDev& wd = J.wins[l];
    const int y = blk % J.emax[1];
    if (y >= wd.E[1]) return;
    const int Ex = wd.E[0], Ey = wd.E[1], Ez = wd.E[2];
    double* sl = sm;            // [x][z] at this y
    double* tx = sm + Ex * Ez;  // T_x
    for (int e = threadIdx.x; e < Ex * Ex; e += blockDim.x) tx[e] = tmat[wd.t_off[0] + e];
    for (int e = threadIdx.x; e < Ex * Ez; e += blockDim.x) {
        const int x = e / Ez, z = e % Ez;
        sl[e] = double(g1[wd.grid_off + (int64_t(x) * Ey + y) * Ez + z]);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < Ex * Ez; e += blockDim.x) {
        const int x = e / Ez, z = e % Ez;
        double acc = 0.0;
        for (int k = 0; k < Ex; ++k) acc += tx[x * Ex + k] * sl[k * Ez + z];
        h[wd.grid_off + (int64_t(x) * Ez + z) * Ey + y] = WT(acc);
    }
}

// 3-feature windows, one work item per wavefront as in the spread. Every lane
// group keeps the same W x W block h(cx + a, cy + b, z .. z + W - 1) (h stored
// as [x][z][y]) for the current layer; per step each group takes one point of
// the layer, lane a forms the share of x-tap a and the W lanes add their shares
// with a fixed xor butterfly.
template <int W, class WT>
__device__ __forceinline__ void gather_grp(const MvJob& J, const int blk) {
    const Segment* __restrict__ segs = J.segs;
    const int32_t* __restrict__ lstart = J.lstart;
    const int32_t* __restrict__ lstart_off = J.lstart_off;
    const WinDev* __restrict__ wins = J.wins;
    const WT* __restrict__ wts = static_cast<const WT*>(J.wts);
    const WT* __restrict__ h = static_cast<const WT*>(J.h);
    const int64_t N = J.N;
    double* __restrict__ fs = J.fs;
    constexpr int G = 64 / W;
    constexpr int REC = rec_stride(W, int(sizeof(WT)));
    constexpr bool kHalf = sizeof(WT) == 8 && W == 8;  // as in the spread
    constexpr int CH = kHalf ? 32 : 64;
    constexpr int PADR = (kHalf ? 32 : 16) / int(sizeof(WT));
    constexpr int RS = REC + PADR;
    constexpr int STEP = CH - G;
    __shared__ __align__(16) WT stw[2][CH * RS];
    const int sid = J.wave_items[J.wave_off[3] + blk];
    const Segment sg = segs[sid];
    const WinDev& wd = wins[sg.win];
    const int lane = threadIdx.x;
    const int g = lane / W, a = lane % W;
    const bool lane_ok = g < G;
    const int64_t base = int64_t(sg.win) * N + sg.start;
    const int32_t* ls = lstart + lstart_off[sid];
    const int cx = sg.col / wd.nb[1];
    const int cy = sg.col % wd.nb[1];
    const int Ey = wd.E[1];
    const WT* hp = h + wd.grid_off + int64_t(cx + (lane_ok ? a : 0)) * wd.E[2] * Ey + cy;
    // hr: the grid values of the current layer's footprint; hn: those of the
    // z-cell the next layer brings in, loaded one layer ahead
    WT hr[W][W], hn[W];
#pragma unroll
    for (int c = 0; c < W; ++c)
#pragma unroll
        for (int b = 0; b < W; ++b) hr[b][c] = hp[int64_t(sg.z0 + c) * Ey + b];
    if (sg.z0 < sg.z1) {
#pragma unroll
        for (int b = 0; b < W; ++b) hn[b] = hp[int64_t(sg.z0 + W) * Ey + b];
    }
    int cc = -1;
    LayerStarts lsw(ls, sg.z1 - sg.z0 + 2, lane);
    stage_records_async<WT, REC, RS, CH>(stw[0], wts, base, 0, sg.count, lane);
    // the first step waits for the first chunk anyway; waiting here as well
    // keeps the layer starts out of the waits inside the loop
    wait_vmem();
    for (int z = sg.z0; z <= sg.z1; ++z) {
        int p, q;
        lsw.get(z - sg.z0, p, q);
        for (int k = p; k < q; k += G) {
            const int c = k / STEP;
            if (c > cc) {
                wait_vmem();
                __syncthreads();
                cc = c;
                if ((c + 1) * STEP < sg.count)
                    stage_records_async<WT, REC, RS, CH>(stw[(c + 1) & 1], wts, base, (c + 1) * STEP, sg.count, lane);
            }
            const int cbase = c * STEP;
            const int pt = k + g;
            const bool act = lane_ok && pt < q;
            double part = 0.0;
            if (act) {
                const WT* w = &stw[c & 1][(pt - cbase) * RS];
                if constexpr (W == 8) {
                    WT wx, wy[W], wz[W];
                    double unused;
                    lds_point8(lds_addr(w + a), lds_addr(w), lds_addr(w + W), wx, unused, wy, wz);
                    WT sy = WT(0);
#pragma unroll
                    for (int b = 0; b < W; ++b) {
                        WT t = WT(0);
#pragma unroll
                        for (int c = 0; c < W; ++c) t += wz[c] * hr[b][c];
                        sy += wy[b] * t;
                    }
                    part = double(wx * sy);
                } else {
                    WT wz[W];
#pragma unroll
                    for (int c = 0; c < W; ++c) wz[c] = w[2 * W + c];
                    WT sy = WT(0);
#pragma unroll
                    for (int b = 0; b < W; ++b) {
                        WT t = WT(0);
#pragma unroll
                        for (int c = 0; c < W; ++c) t += wz[c] * hr[b][c];
                        sy += w[W + b] * t;
                    }
                    part = double(w[a] * sy);
                }
            }
            if constexpr ((W & (W - 1)) == 0) {
#pragma unroll
                for (int o = W / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
            } else {
                double tot = 0.0;
#pragma unroll
                for (int q2 = 0; q2 < W; ++q2) tot += __shfl(part, g * W + q2, 64);
                part = tot;
            }
            if (act && a == 0) fs[base + pt] = part;
        }
        if (z < sg.z1) {
#pragma unroll
            for (int b = 0; b < W; ++b) {
#pragma unroll
                for (int c = 0; c < W - 1; ++c) hr[b][c] = hr[b][c + 1];
                hr[b][W - 1] = hn[b];
            }
            if (z + 1 < sg.z1) {
#pragma unroll
                for (int b = 0; b < W; ++b) hn[b] = hp[int64_t(z + 1 + W) * Ey + b];
            }
        }
    }
}

// 1- and 2-feature windows: one lane per work item.
template <int W, int WY, class WT>
__device__ __forceinline__ void gather_lane(const MvJob& J, const int blk) {
    const Segment* __restrict__ segs = J.segs;
    const WinDev* __restrict__ wins = J.wins;
    const int32_t* __restrict__ zq = J.zq;
    const WT* __restrict__ wts = static_cast<const WT*>(J.wts);
    const WT* __restrict__ h = static_cast<const WT*>(J.h);
    const int64_t N = J.N;
    double* __restrict__ fs = J.fs;
    const int sid = J.wave_items[J.wave_off[WY == 1 ? 1 : 2] + blk * 64 + threadIdx.x];
    if (sid < 0) return;
    const Segment sg = segs[sid];
    const WinDev& wd = wins[sg.win];
    const int cx = sg.col / wd.nb[1];
    const int cy = sg.col % wd.nb[1];
    const int Ey = wd.E[1];
    const WT* hp = h + wd.grid_off + int64_t(cx) * wd.E[2] * Ey + cy;
    const int64_t base = int64_t(sg.win) * N + sg.start;
    WT hr[WY][W];
    int zr = sg.z0;
#pragma unroll
    for (int c = 0; c < W; ++c)
#pragma unroll
        for (int b = 0; b < WY; ++b) hr[b][c] = hp[int64_t(zr + c) * Ey + b];
    for (int k = 0; k < sg.count; ++k) {
        const int64_t gi = base + k;
        const int zj = zq[gi];
        while (zr < zj) {
#pragma unroll
            for (int b = 0; b < WY; ++b) {
#pragma unroll
                for (int c = 0; c < W - 1; ++c) hr[b][c] = hr[b][c + 1];
                hr[b][W - 1] = hp[int64_t(zr + W) * Ey + b];
            }
            ++zr;
        }
        const WT* w = wts + gi * rec_stride(W, int(sizeof(WT)));
        WT sy = WT(0);
#pragma unroll
        for (int b = 0; b < WY; ++b) {
            WT t = WT(0);
#pragma unroll
            for (int c = 0; c < W; ++c) t += w[2 * W + c] * hr[b][c];
            sy += w[W + b] * t;
        }
        fs[gi] = double(sy);
    }
}

// Gathering of every window in one launch, in the order of the spreading
template <int W, class WT>
__global__ __launch_bounds__(64) void k_gather(const MvLaunch ML) {
    int blk = blockIdx.x;
    const MvJob& J = ML.job[job_of(ML, blk)];
    if (blk < J.nwave[3])
        gather_grp<W, WT>(J, blk);
    else if (blk < J.nwave[3] + J.nwave[2])
        gather_lane<W, W, WT>(J, blk - J.nwave[3]);
    else
        gather_lane<W, 1, WT>(J, blk - J.nwave[3] - J.nwave[2]);
}

__global__ void k_window_sum(const MvLaunch ML) {
    int blk = blockIdx.x;
    const MvJob& J = ML.job[job_of(ML, blk)];
    const int64_t i = blk * (int64_t)blockDim.x + threadIdx.x;
    const int64_t N = J.N;
    if (i >= N) return;
    double acc = 0.0;
    for (int l = 0; l < J.P; ++l) acc += J.wins[l].eta * J.fs[int64_t(l) * N + J.pos[int64_t(l) * N + i]];
    J.y[i] = acc;
}

MvJob make_job(Plan& pl, const double* x, double* y) {
    MvJob J;
    std::memset(&J, 0, sizeof(J));
    const bool f64 = pl.precision == ANOVA_PREC_FP64;
    J.x = x;
    J.y = y;
    J.perm = pl.perm.p;
    J.pos = pl.pos.p;
    J.zq = pl.zq.p;
    J.wts = f64 ? static_cast<const void*>(pl.wts64.p) : static_cast<const void*>(pl.wts32.p);
    J.segs = pl.segs.p;
    J.lstart = pl.lstart.p;
    J.lstart_off = pl.lstart_off.p;
    J.wins = pl.wins_d.p;
    J.alone = pl.alone.p;
    J.wave_items = pl.wave_items.p;
    J.flist = pl.flist.p;
    J.fold = pl.fold.p;
    J.sbase = pl.sbase.p;
    J.crange = pl.crange.p;
    J.tmat = pl.tmat.p;
    J.vs = pl.vs.p;
    J.fs = pl.fs.p;
    J.slab = f64 ? static_cast<void*>(pl.slab64.p) : static_cast<void*>(pl.slab32.p);
    J.g = f64 ? static_cast<void*>(pl.g64.p) : static_cast<void*>(pl.g32.p);
    J.h = f64 ? static_cast<void*>(pl.h64.p) : static_cast<void*>(pl.h32.p);
    J.ca = f64 ? static_cast<void*>(pl.c64a.p) : static_cast<void*>(pl.c32a.p);
    J.N = pl.N;
    J.nflist = pl.nflist;
    J.nflist3 = pl.nflist3;
    for (int k = 0; k < 4; ++k) {
        J.wave_off[k] = pl.wave_off[k];
        J.nwave[k] = pl.nwave[k];
    }
    J.P = pl.P;
    for (int a = 0; a < 3; ++a) J.emax[a] = pl.emax[a];
    return J;
}

// Launches kernel `kern` over the jobs of L with blocks(job) blocks each (jobs
// with none are skipped by the offsets); returns false if no job has work.
template <class F, class K>
bool launch_jobs(MvLaunch& L, F blocks, K kern, unsigned threads, size_t lds, hipStream_t st) {
    int64_t tot = 0;
    for (int j = 0; j < L.njobs; ++j) {
        L.off[j] = int32_t(tot);
        tot += blocks(L.job[j]);
    }
    L.off[L.njobs] = int32_t(tot);
    if (tot == 0) return false;
    ANV_CHECK(tot < (int64_t(1) << 31), "launch too large");
    hipLaunchKernelGGL(kern, dim3(unsigned(tot)), dim3(threads), lds, st, L);
    return true;
}

template <int W, class WT>
void run_jobs(MvLaunch& L, Plan* prof, hipStream_t st) {
    auto ev = [&]() {
        if (prof && prof->profiling) prof->record_stage_event(st);
    };
    int e0 = 1, e1 = 1, e2 = 1;
    for (int j = 0; j < L.njobs; ++j) {
        e0 = std::max(e0, L.job[j].emax[0]);
        e1 = std::max(e1, L.job[j].emax[1]);
        e2 = std::max(e2, L.job[j].emax[2]);
    }
    ev();
    launch_jobs(L, [](const MvJob& J) { return int64_t(nblocks(J.N * J.P)); }, k_permute, kThreads, 0, st);
    ev();
    launch_jobs(L, [](const MvJob& J) { return int64_t(J.nwave[3]) + J.nwave[2] + J.nwave[1]; }, k_spread<W, WT>, 64, 0,
                st);
    ev();
    launch_jobs(L, [](const MvJob& J) { return (J.nflist3 + 3) / 4; }, k_fold_cols<WT>, 256, 0, st);
    launch_jobs(L, [](const MvJob& J) { return J.nflist - J.nflist3; }, k_fold_cols_wide<WT>, 256, 0, st);
    ev();
    launch_jobs(L, [](const MvJob& J) { return int64_t(J.emax[0]) * J.P; }, k_fold_conv_yz<W, WT>, fold_conv1_threads<WT>(),
                size_t(2 * e1 * e2 + e1 * e1 + e2 * e2) * sizeof(double), st);
    launch_jobs(L, [](const MvJob& J) { return int64_t(J.emax[1]) * J.P; }, k_conv_x<WT>, 256,
                size_t(e0 * e2 + e0 * e0) * sizeof(double), st);
    ev();
    launch_jobs(L, [](const MvJob& J) { return int64_t(J.nwave[3]) + J.nwave[2] + J.nwave[1]; }, k_gather<W, WT>, 64, 0,
                st);
    ev();
    launch_jobs(L, [](const MvJob& J) { return int64_t(nblocks(J.N)); }, k_window_sum, kThreads, 0, st);
    ev();
    ANV_HIP(hipGetLastError());
}

void run_launch(MvLaunch& L, int W, int precision, Plan* prof, hipStream_t st) {
    const bool f64 = precision == ANOVA_PREC_FP64;
    switch (W) {
        case 4: f64 ? run_jobs<4, double>(L, prof, st) : run_jobs<4, float>(L, prof, st); break;
        case 6: f64 ? run_jobs<6, double>(L, prof, st) : run_jobs<6, float>(L, prof, st); break;
        case 8: f64 ? run_jobs<8, double>(L, prof, st) : run_jobs<8, float>(L, prof, st); break;
        default: throw Error(ANOVA_INVALID_ARG, "unsupported cutoff");
    }
}

}  // namespace

void Plan::record_stage_event(hipStream_t st) {
    if (events_used == events.size()) {
        hipEvent_t e;
        ANV_HIP(hipEventCreate(&e));
        events.push_back(e);
    }
    ANV_HIP(hipEventRecord(events[events_used++], st));
}

Plan::~Plan() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
}

void profile_begin(Plan& pl) {
    pl.profiling = true;
    pl.events_used = 0;
}

int profile_end(Plan& pl, double* stage_ms, int nstage) {
    pl.profiling = false;
    const size_t per = ANOVA_NSTAGES + 1;
    const size_t passes = pl.events_used / per;
    std::vector<double> acc(ANOVA_NSTAGES, 0.0);
    if (passes > 0) ANV_HIP(hipEventSynchronize(pl.events[passes * per - 1]));
    for (size_t p = 0; p < passes; ++p)
        for (int s = 0; s < ANOVA_NSTAGES; ++s) {
            float ms = 0.f;
            ANV_HIP(hipEventElapsedTime(&ms, pl.events[p * per + s], pl.events[p * per + s + 1]));
            acc[s] += ms;
        }
    for (int s = 0; s < nstage && s < ANOVA_NSTAGES; ++s) stage_ms[s] = passes ? acc[s] / passes : 0.0;
    pl.events_used = 0;
    return int(passes);
}

void enqueue_matvec(Plan& pl, const double* x, int R, int64_t ldx, double* y, int64_t ldy,
                    hipStream_t st) {
    if (pl.batch_min_rhs > 0 && R >= pl.batch_min_rhs && batched_supported(pl)) {
        enqueue_matvec_batched(pl, x, R, ldx, y, ldy, st);
        return;
    }
    MvLaunch L;
    L.njobs = 1;
    for (int r = 0; r < R; ++r) {
        L.job[0] = make_job(pl, x + int64_t(r) * ldx, y + int64_t(r) * ldy);
        run_launch(L, pl.W, pl.precision, &pl, st);
    }
}

// ---------------------------------------------------------------- allocation-free matvec
// Scratch of enqueue_matvec_noalloc: one array per device, allocated with the
// code object when the library is loaded on the device and held until the
// process ends. Host code never passes `scratch` itself to a kernel (in host
// code the name is a host-side stand-in, not a device address): it uses the
// device address that hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the first call
// on the device, with that device current).
unsigned char* noalloc_scratch() {
    int dev = 0;
    ANV_HIP(hipGetDevice(&dev));
    ANV_CHECK(dev >= 0 && dev < kMaxDevices, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        ANV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        ANV_CHECK(p != nullptr, "no device address for the scratch array");
        g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
    }
    return g_scratch_ptr[dev];
}

// Byte offsets of the one-vector matvec's scratch arrays inside the scratch
// region (each 256-byte aligned): vs, fs, slab, g, h, fold target; [6] = total.
void noalloc_layout(const Plan& pl, size_t (&off)[7]) {
    const size_t elem = pl.precision == ANOVA_PREC_FP64 ? sizeof(double) : sizeof(float);
    const size_t np = size_t(pl.N) * size_t(pl.P);
    const size_t bytes[6] = {(np + 2) * sizeof(double), np * sizeof(double), size_t(std::max<int64_t>(pl.slab_total, 1)) * elem,
                             size_t(pl.grid_total) * elem, size_t(pl.grid_total) * elem,
                             size_t(std::max<int64_t>(pl.tgt_total, 1)) * elem};
    size_t o = 0;
    for (int k = 0; k < 6; ++k) {
        off[k] = o;
        o += (bytes[k] + 255) & ~size_t(255);
    }
    off[6] = o;
}

}  // namespace

size_t noalloc_scratch_bytes(const Plan& pl) {
    size_t off[7];
    noalloc_layout(pl, off);
    return off[6];
}

void enqueue_matvec_noalloc(Plan& pl, const double* x, int R, int64_t ldx, double* y, int64_t ldy, hipStream_t st) {
    size_t off[7];
    noalloc_layout(pl, off);
    if (off[6] > kNoAllocScratchBytes)
        throw Error(ANOVA_INVALID_ARG, "plan needs " + std::to_string(off[6]) +
                                           " bytes of matvec scratch, more than the allocation-free maximum of " +
                                           std::to_string(kNoAllocScratchBytes) + " bytes");
    unsigned char* base = noalloc_scratch();
    MvLaunch L;
    L.njobs = 1;
    for (int r = 0; r < R; ++r) {
        MvJob J = make_job(pl, x + int64_t(r) * ldx, y + int64_t(r) * ldy);
        J.vs = reinterpret_cast<double*>(base + off[0]);
        J.fs = reinterpret_cast<double*>(base + off[1]);
        J.slab = base + off[2];
        J.g = base + off[3];
        J.h = base + off[4];
        J.ca = base + off[5];
        L.job[0] = J;
        run_launch(L, pl.W, pl.precision, nullptr, st);
    }
}

void enqueue_matvec_multi(Plan* const* plans, const double* const* x, double* const* y, int n, hipStream_t st) {
    // one launch per stage for up to kMaxJobs plans of equal cutoff and precision
    std::vector<int> done(n, 0);
    for (int i = 0; i < n; ++i) {
        if (done[i]) continue;
        MvLaunch L;
        L.njobs = 0;
        for (int k = i; k < n && L.njobs < kMaxJobs; ++k) {
            if (done[k] || plans[k]->W != plans[i]->W || plans[k]->precision != plans[i]->precision) continue;
            bool dup = false;
            for (int q = 0; q < L.njobs; ++q) dup |= (plans[k]->pos.p == L.job[q].pos);
            if (dup) continue;  // a plan's scratch serves one vector per launch
            L.job[L.njobs++] = make_job(*plans[k], x[k], y[k]);
            done[k] = 1;
        }
        run_launch(L, plans[i]->W, plans[i]->precision, nullptr, st);
    }
}

}  // namespace anv
