// Batched ANOVA-NFFT matvec: 16 right-hand sides per pass, FP32 grids and
// weights, FP64 window sums (mixed precision). Same algorithm and the same
// fixed summation orders as the single-vector path (matvec.hip); every array of
// partial sums carries the 16 right-hand sides as its innermost index.
//
// For 3-feature windows (2m = 8 taps per axis) spreading and gathering are
// dense contractions over the points of one grid layer and run on the matrix
// cores (v_mfma_f32_16x16x4_f32):
//   spread: T[(a, r)][(b, c)] += sum_p (v_{p,r} wx_p[a]) (wy_p[b] wz_p[c - z_p])
//           M = 8 x-taps x 16 rhs, N = 8 y-taps x 8 z-cells, K = 4 points;
//   gather: S[(a, r)][p] = sum_{(b,c)} h_r(a, b, c) (wy_p[b] wz_p[c - z_p]),
//           f_{p,r} = sum_a wx_p[a] S[(a, r)][p]; M = 128, N = 16 points, K = 64.
// The z-cells form a ring of 8 physical columns (cell z lives in column z & 7),
// so advancing a layer is a flush (spread) or reload (gather) of one column.
#include "plan.hpp"

namespace anv {

namespace {

constexpr int RB = 16;  // right-hand sides per pass
constexpr int kT = 256;
inline unsigned nblk(int64_t n, int t = kT) { return unsigned(std::max<int64_t>(1, (n + t - 1) / t)); }

typedef float f4 __attribute__((ext_vector_type(4)));
// four consecutive values of the element type, moved as one vector access
template <class T> struct Vec4;
template <> struct Vec4<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec4<double> { typedef double type __attribute__((ext_vector_type(4))); };
template <class T> using v4 = typename Vec4<T>::type;

__device__ inline void wait_vmem_b() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

__device__ inline void dma16(const void* src, void* lds) {
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                     (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}

// Column pointers of one pass: right-hand side r is read from x[r] and its
// result written to y[r] (N doubles each); columns r >= R are absent.
struct ColPtrs {
    const double* x[RB];
    double* y[RB];
};

// xt[i][r] = x_r[i] in the pass's element type (zero for r >= R); 64 points per
// block, transposed through LDS so that both the reads and the writes are
// coalesced. Also resets the spread and gather work queues of the pass.
template <class T>
__global__ __launch_bounds__(256) void k_transpose_in(const ColPtrs cols, int R, int64_t N, T* __restrict__ xt,
                                                      int32_t* __restrict__ queues) {
    __shared__ T s[RB][65];
    if (blockIdx.x == 0 && threadIdx.x < 2) queues[threadIdx.x] = 0;  // work queues of this pass
    const int64_t i0 = int64_t(blockIdx.x) * 64;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = j * 256 + threadIdx.x;
        const int r = e / 64, i = e % 64;  // r is uniform across a wavefront
        s[r][i] = (r < R && i0 + i < N) ? T(cols.x[r][i0 + i]) : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = j * 256 + threadIdx.x;
        const int i = e / RB, r = e % RB;
        if (i0 + i < N) xt[(i0 + i) * RB + r] = s[r][i];
    }
}

// LDS chunks of CHB = 32 consecutive points of a work item, moved by DMA (16
// bytes per lane per instruction). A record occupies RPB = 36 floats: x taps,
// y taps, z taps, and the z taps again, so that any 8 cyclically consecutive z
// taps are 8 consecutive floats, then 4 floats of padding, so that records of
// consecutive points start 36 words apart and the 16 points a step reads at the
// same offset fall on different LDS banks. Slot s (16 bytes) of a chunk holds
// piece s % 9 of record s / 9. A value row holds the point's 16 right-hand
// sides. Slots past the item read its last point (finite data; callers mask).
constexpr int CHB = 32;
constexpr int RPB = 36;

__device__ inline void stage_records(float* lrec, const float* __restrict__ wts, int64_t base, int cstart, int count,
                                     int lane) {
    const float* ub = wts + (base + cstart) * 24;  // uniform; lanes add small offsets
    const int last = count - 1 - cstart;
    constexpr int NS = CHB * RPB / 4;  // 16-byte slots of a chunk: 288, four 1 KB instructions and a half one
#pragma unroll
    for (int j = 0; j < (NS + 63) / 64; ++j) {
        const int sl = j * 64 + lane;
        if (sl < NS) {
            const int rec = sl / (RPB / 4), piece = sl % (RPB / 4);
            const int e = piece < 8 ? 4 * piece : 0;
            dma16(ub + min(rec, last) * 24 + (e < 24 ? e : e - 8), lrec + j * 256);
        }
    }
}

// Point indices of the two value rows a lane moves for the chunk starting at
// cstart (rows past the item repeat its last point).
__device__ inline void value_rows(const int32_t* __restrict__ perm, int64_t base, int cstart, int count, int lane,
                                  int32_t (&pr)[2]) {
    const int last = count - 1 - cstart;
#pragma unroll
    for (int j = 0; j < 2; ++j) pr[j] = perm[base + cstart + min(j * 16 + lane / 4, last)];
}

// The 16 right-hand sides of those points, gathered from the point-major input
// straight into LDS (16 rows per 1 KB instruction).
__device__ inline void stage_values(float* lval, const float* __restrict__ xt, const int32_t (&pr)[2], int lane) {
#pragma unroll
    for (int j = 0; j < 2; ++j) dma16(xt + int64_t(pr[j]) * RB + (lane % 4) * 4, lval + j * 256);
}

// LDS byte address of a pointer into shared memory (the low half of its flat address)
__device__ inline uint32_t lds_addr(const void* p) { return static_cast<uint32_t>(reinterpret_cast<uintptr_t>(p)); }

// Reads of staged chunk data. They are written as asm with the wait for their
// own completion inside the block: the compiler would otherwise make every LDS
// read wait for all DMA in flight, including the prefetch of the next chunk.
// Chunk data are only read after the explicit wait at the chunk switch.
__device__ inline void lds_spread_operands(uint32_t rec, uint32_t ywy, uint32_t ywz, uint32_t yv, f4& wx0, f4& wx1,
                                           f4& wy, float& wz, float& v) {
    asm volatile(
        "ds_read_b128 %0, %5\n\t"
        "ds_read_b128 %1, %5 offset:16\n\t"
        "ds_read_b128 %2, %6\n\t"
        "ds_read_b32 %3, %7\n\t"
        "ds_read_b32 %4, %8\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(wx0), "=&v"(wx1), "=&v"(wy), "=&v"(wz), "=&v"(v)
        : "v"(rec), "v"(ywy), "v"(ywz), "v"(yv)
        : "memory");
}

__device__ inline void lds_gather_operands(uint32_t rec, uint32_t ywy, uint32_t ywz, f4& wx0, f4& wx1, float& wy0,
                                           float& wy1, float (&wz)[8]) {
    asm volatile(
        "ds_read_b128 %0, %12\n\t"
        "ds_read_b128 %1, %12 offset:16\n\t"
        "ds_read_b32 %2, %13\n\t"
        "ds_read_b32 %3, %13 offset:16\n\t"
        "ds_read_b32 %4, %14\n\t"
        "ds_read_b32 %5, %14 offset:4\n\t"
        "ds_read_b32 %6, %14 offset:8\n\t"
        "ds_read_b32 %7, %14 offset:12\n\t"
        "ds_read_b32 %8, %14 offset:16\n\t"
        "ds_read_b32 %9, %14 offset:20\n\t"
        "ds_read_b32 %10, %14 offset:24\n\t"
        "ds_read_b32 %11, %14 offset:28\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(wx0), "=&v"(wx1), "=&v"(wy0), "=&v"(wy1), "=&v"(wz[0]), "=&v"(wz[1]), "=&v"(wz[2]), "=&v"(wz[3]),
          "=&v"(wz[4]), "=&v"(wz[5]), "=&v"(wz[6]), "=&v"(wz[7])
        : "v"(rec), "v"(ywy), "v"(ywz)
        : "memory");
}

__device__ inline void lds_store_f4(uint32_t addr, f4 v) {
    asm volatile("ds_write_b128 %0, %1" : : "v"(addr), "v"(v) : "memory");
}

__device__ inline void lds_wait() { asm volatile("s_waitcnt lgkmcnt(0)" : : : "memory"); }

__device__ inline f4 lds_load_f4(uint32_t addr) {
    f4 v;
    asm volatile("ds_read_b128 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=&v"(v) : "v"(addr) : "memory");
    return v;
}

// ---------------------------------------------------------------- spread (3 features, MFMA)
// Lane = 16 lk + lr. Accumulator tile (mb, nb): rows (x tap a = mb, rhs r),
// columns n = lr -> (y tap b = nb + 4 (lr / 8), physical z column lr % 8); the
// lane holds rows r = 4 lk .. 4 lk + 3 of column lr. A step takes the points
// k .. k+3 of one layer, point k + lk being k-index lk of the contraction.
// Chunk c of the staged data serves the steps that start in [c STEP, (c+1) STEP).
__global__ __launch_bounds__(64) void k_spread_mfma(const int32_t* __restrict__ wave_items, int32_t nitems,
                                                    int32_t* __restrict__ queue,
                                                    const Segment* __restrict__ segs,
                                                    const int32_t* __restrict__ lstart,
                                                    const int32_t* __restrict__ lstart_off,
                                                    const WinDev* __restrict__ wins,
                                                    const uint8_t* __restrict__ alone,
                                                    const float* __restrict__ wts,
                                                    const int32_t* __restrict__ perm,
                                                    const float* __restrict__ xt, int64_t N,
                                                    float* __restrict__ slab, float* __restrict__ tgt) {
    constexpr int STEP = CHB - 4;
    __shared__ __align__(16) float srec[2][CHB * RPB];
    __shared__ __align__(16) float sval[2][CHB * RB];
    __shared__ __align__(16) float stg[64 * RB];
    const int lane = threadIdx.x;
    // work items are taken in order (longest first) from a queue shared by the
    // resident wavefronts, so that the matrix-core work evens out over the SIMDs
    for (;;) {
        int it = 0;
        if (lane == 0) it = atomicAdd(queue, 1);
        it = __builtin_amdgcn_readfirstlane(it);
        if (it >= nitems) break;
        const int sid = wave_items[it];
        const Segment sg = segs[sid];
        const WinDev& wd = wins[sg.win];
        const int lr = lane & 15, lk = lane >> 4;
        const int64_t base = int64_t(sg.win) * N + sg.start;
        const int32_t* ls = lstart + lstart_off[sid];
        const bool direct = alone[sid] != 0;
        const int cx = sg.col / wd.nb[1], cy = sg.col % wd.nb[1];
        const int E1 = wd.E[1], E2 = wd.E[2];
        // Output element of footprint position (a, b) at layer L, as U(L) + a SA + b SB:
        // fold target tgt[tgt_off + (((cx + a) E1 + cy + b) 64 + 8 a + b) E2 + L][r] for
        // an item alone in its column, else its slab row [L - z0][8 a + b][r]
        const int64_t SA = direct ? int64_t(64 * E1 + 8) * E2 : 8;
        const int64_t SB = direct ? int64_t(65) * E2 : 1;
        const int64_t U0 = direct ? wd.tgt_off + (int64_t(cx) * E1 + cy) * 64 * E2 : sg.off - int64_t(sg.z0) * 64;
        const int64_t UL = direct ? 1 : 64;
        float* const outp = direct ? tgt : slab;
        f4 acc[32];
#pragma unroll
        for (int t = 0; t < 32; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
        // Write z cell `layer` and clear it. Its values sit in the lanes with
        // lr % 8 == layer % 8; they go through LDS (rows [8 a + b][r]) so that
        // the global stores are whole-wavefront: four lanes per 64-byte row.
        const uint32_t stg0 = lds_addr(&stg[0]);
        auto flush = [&](int layer) __attribute__((always_inline)) {
            if ((lr & 7) == (layer & 7)) {
#pragma unroll
                for (int mb = 0; mb < 8; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb) {
                        const int ab = mb * 8 + nb + 4 * (lr >> 3);
                        lds_store_f4(stg0 + uint32_t(ab * RB + 4 * lk) * 4, acc[mb * 4 + nb]);
                        acc[mb * 4 + nb] = f4{0.f, 0.f, 0.f, 0.f};
                    }
            }
            lds_wait();
            __syncthreads();
            float* const row = outp + (U0 + int64_t(layer) * UL) * RB + 4 * (lane & 3);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ab = 16 * j + (lane >> 2);
                const f4 v = lds_load_f4(stg0 + uint32_t(ab * RB + 4 * (lane & 3)) * 4);
                *reinterpret_cast<f4*>(row + ((ab >> 3) * SA + (ab & 7) * SB) * RB) = v;
            }
        };
        const uint32_t rec0 = lds_addr(&srec[0][0]), val0 = lds_addr(&sval[0][0]);
        constexpr uint32_t RECB = CHB * RPB * 4, VALB = CHB * RB * 4;  // bytes per buffer
        int cc = -1;
        int32_t prow[2];  // value rows of the next chunk to stage, loaded a chunk ahead
        stage_records(srec[0], wts, base, 0, sg.count, lane);
        value_rows(perm, base, 0, sg.count, lane, prow);
        stage_values(sval[0], xt, prow, lane);
        if (STEP < sg.count) value_rows(perm, base, STEP, sg.count, lane, prow);
        for (int z = sg.z0; z <= sg.z1; ++z) {
            const int p = ls[z - sg.z0], q = ls[z - sg.z0 + 1];
            for (int k = p; k < q; k += 4) {
                const int c = k / STEP;
                if (c > cc) {  // chunk c has landed (and earlier stores have drained); prefetch c + 1
                    wait_vmem_b();
                    __syncthreads();
                    cc = c;
                    if ((c + 1) * STEP < sg.count) {
                        stage_records(srec[(c + 1) & 1], wts, base, (c + 1) * STEP, sg.count, lane);
                        stage_values(sval[(c + 1) & 1], xt, prow, lane);
                        if ((c + 2) * STEP < sg.count) value_rows(perm, base, (c + 2) * STEP, sg.count, lane, prow);
                    }
                }
                const int pt = k + lk;
                const uint32_t slot = uint32_t(pt - c * STEP);
                const uint32_t rb = rec0 + uint32_t(c & 1) * RECB + slot * (RPB * 4);
                f4 wx0, wx1, wy;
                float wz, v;
                lds_spread_operands(rb, rb + 32 + 16 * uint32_t(lr >> 3), rb + 64 + 4 * uint32_t((lr - z) & 7),
                                    val0 + uint32_t(c & 1) * VALB + (slot * RB + lr) * 4, wx0, wx1, wy, wz, v);
                v = pt < q ? v : 0.0f;
                const float bv[4] = {wy[0] * wz, wy[1] * wz, wy[2] * wz, wy[3] * wz};
                const float av[8] = {v * wx0[0], v * wx0[1], v * wx0[2], v * wx0[3],
                                     v * wx1[0], v * wx1[1], v * wx1[2], v * wx1[3]};
    #pragma unroll
                for (int mb = 0; mb < 8; ++mb)
    #pragma unroll
                    for (int nb = 0; nb < 4; ++nb)
                        acc[mb * 4 + nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mb], bv[nb], acc[mb * 4 + nb], 0, 0, 0);
            }
            flush(z);
        }
        for (int j = 1; j < 8; ++j) flush(sg.z1 + j);
    }
}

// ---------------------------------------------------------------- gather (3 features, MFMA)
// S[(a, r)][p] = sum_K H[(a, r)][K] B[K][p] over the 64 taps K <-> (y tap b, z
// column c); m-block mb is x tap a; a step takes the 16 points k .. k+15 of one
// layer (column lr of B and of S). The contraction runs on
// v_mfma_f32_16x16x32_bf16 with every FP32 operand split into bf16 hi + lo
// parts: H B ~ Hhi Bhi + Hhi Blo + Hlo Bhi (the dropped lo*lo term is below
// 2^-16 of each product; sums stay in FP32). In k-step ks2 lane (lr, lk) holds
// the 8 taps (b = 4 ks2 + lk, c = j), j = 0..7, i.e. one tap of every z column,
// so refilling a column after a layer touches one element in every lane. The
// ring holds layer z0 + ((c - z0) mod 8) in column c; after layer z the column
// z mod 8 takes layer z + 8 from registers loaded a layer ahead.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

__global__ __launch_bounds__(64, 2) void k_gather_mfma(const int32_t* __restrict__ wave_items, int32_t nitems,
                                                    int32_t* __restrict__ queue,
                                                    const Segment* __restrict__ segs,
                                                    const int32_t* __restrict__ lstart,
                                                    const int32_t* __restrict__ lstart_off,
                                                    const WinDev* __restrict__ wins,
                                                    const float* __restrict__ wts,
                                                    const float* __restrict__ h, int64_t N,
                                                    float* __restrict__ fs) {
    constexpr int STEP = CHB - 16;
    __shared__ __align__(16) float srec[2][CHB * RPB];
    const int lane = threadIdx.x;
    // work items are taken in order (longest first) from a queue shared by the
    // resident wavefronts, so that the matrix-core work evens out over the SIMDs
    for (;;) {
        int it = 0;
        if (lane == 0) it = atomicAdd(queue, 1);
        it = __builtin_amdgcn_readfirstlane(it);
        if (it >= nitems) break;
        const int sid = wave_items[it];
        const Segment sg = segs[sid];
        const WinDev& wd = wins[sg.win];
        const int lr = lane & 15, lk = lane >> 4;
        const int64_t base = int64_t(sg.win) * N + sg.start;
        const int32_t* ls = lstart + lstart_off[sid];
        const int cx = sg.col / wd.nb[1], cy = sg.col % wd.nb[1];
        const int Ey = wd.E[1], Ez = wd.E[2];
        // h[x][z][y][r]: grid cell (cx + a, cy + b, layer), rhs lr
        const float* hp = h + (wd.grid_off + int64_t(cx) * Ez * Ey + cy) * RB + lr;
        bf8 Hh[8][2], Hl[8][2];
#pragma unroll
        for (int ks2 = 0; ks2 < 2; ++ks2)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int layer = sg.z0 + ((j - sg.z0) & 7);
#pragma unroll
                for (int mb = 0; mb < 8; ++mb) {
                    __bf16 hi, lo;
                    split_bf16(hp[((int64_t(mb) * Ez + layer) * Ey + 4 * ks2 + lk) * RB], hi, lo);
                    Hh[mb][ks2][j] = hi;
                    Hl[mb][ks2][j] = lo;
                }
            }
        float pre[8][2];
        if (sg.z0 < sg.z1) {
#pragma unroll
            for (int mb = 0; mb < 8; ++mb)
#pragma unroll
                for (int ks2 = 0; ks2 < 2; ++ks2) pre[mb][ks2] = hp[((int64_t(mb) * Ez + sg.z0 + 8) * Ey + 4 * ks2 + lk) * RB];
        }
        const uint32_t rec0 = lds_addr(&srec[0][0]);
        constexpr uint32_t RECB = CHB * RPB * 4;
        int cc = -1;
        stage_records(srec[0], wts, base, 0, sg.count, lane);
        for (int z = sg.z0; z <= sg.z1; ++z) {
            const int p = ls[z - sg.z0], q = ls[z - sg.z0 + 1];
            for (int k = p; k < q; k += 16) {
                const int c = k / STEP;
                if (c > cc) {
                    wait_vmem_b();
                    __syncthreads();
                    cc = c;
                    if ((c + 1) * STEP < sg.count) stage_records(srec[(c + 1) & 1], wts, base, (c + 1) * STEP, sg.count, lane);
                }
                const int pt = k + lr;
                const uint32_t rb = rec0 + uint32_t(c & 1) * RECB + uint32_t(pt - c * STEP) * (RPB * 4);
                f4 wx0, wx1;
                float wy0, wy1, wzr[8];  // wzr[c]: z tap of the ring cell in column c
                lds_gather_operands(rb, rb + 32 + 4 * uint32_t(lk), rb + 64 + 4 * uint32_t((-z) & 7), wx0, wx1, wy0, wy1,
                                    wzr);
                bf8 Bh[2], Bl[2];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    __bf16 hi, lo;
                    split_bf16(wy0 * wzr[j], hi, lo);
                    Bh[0][j] = hi;
                    Bl[0][j] = lo;
                    split_bf16(wy1 * wzr[j], hi, lo);
                    Bh[1][j] = hi;
                    Bl[1][j] = lo;
                }
                f4 D[8];
#pragma unroll
                for (int mb = 0; mb < 8; ++mb) D[mb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks2 = 0; ks2 < 2; ++ks2)
#pragma unroll
                    for (int mb = 0; mb < 8; ++mb) D[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Hh[mb][ks2], Bh[ks2], D[mb], 0, 0, 0);
#pragma unroll
                for (int ks2 = 0; ks2 < 2; ++ks2)
#pragma unroll
                    for (int mb = 0; mb < 8; ++mb) D[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Hh[mb][ks2], Bl[ks2], D[mb], 0, 0, 0);
#pragma unroll
                for (int ks2 = 0; ks2 < 2; ++ks2)
#pragma unroll
                    for (int mb = 0; mb < 8; ++mb) D[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Hl[mb][ks2], Bh[ks2], D[mb], 0, 0, 0);
                if (pt < q) {  // the lane holds S[(a, r = 4 lk + i)][point lr]
                    f4 f = wx0[0] * D[0];
                    f += wx0[1] * D[1];
                    f += wx0[2] * D[2];
                    f += wx0[3] * D[3];
                    f += wx1[0] * D[4];
                    f += wx1[1] * D[5];
                    f += wx1[2] * D[6];
                    f += wx1[3] * D[7];
                    *reinterpret_cast<f4*>(fs + (base + pt) * RB + 4 * lk) = f;
                }
            }
            if (z < sg.z1) {  // column z mod 8 takes layer z + 8; load layer z + 9 for the next column
                switch (z & 7) {
#define ANV_REFILL(J)                                          \
    case J:                                                    \
        _Pragma("unroll") for (int mb = 0; mb < 8; ++mb)       \
            _Pragma("unroll") for (int ks2 = 0; ks2 < 2; ++ks2) { \
                __bf16 hi, lo;                                 \
                split_bf16(pre[mb][ks2], hi, lo);              \
                Hh[mb][ks2][J] = hi;                           \
                Hl[mb][ks2][J] = lo;                           \
            }                                                  \
        break;
                    ANV_REFILL(0) ANV_REFILL(1) ANV_REFILL(2) ANV_REFILL(3)
                    ANV_REFILL(4) ANV_REFILL(5) ANV_REFILL(6) ANV_REFILL(7)
#undef ANV_REFILL
                }
                if (z + 1 < sg.z1) {
#pragma unroll
                    for (int mb = 0; mb < 8; ++mb)
#pragma unroll
                        for (int ks2 = 0; ks2 < 2; ++ks2)
                            pre[mb][ks2] = hp[((int64_t(mb) * Ez + z + 9) * Ey + 4 * ks2 + lk) * RB];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- FP64 spread and gather (3 features, MFMA)
// The FP64 path runs the same contractions on v_mfma_f64_16x16x4f64 with FP64
// records, inputs, grids and sums. Its accumulators and grid tiles take twice
// the registers of the FP32 ones, so a wavefront takes one half of the 16
// right-hand sides: M = 8 x taps x 8 rhs. A work item (segment) goes to a block
// of two wavefronts, one per half, which stage each chunk of point records into
// LDS once for both (each wavefront moves half of the chunk's DMA slots) and
// run the same loops in step, so that the block barriers line up.
// Operand layouts as for the FP32 instruction (A: lane (i, k), B: lane (k, j)),
// but the result row of register v in lane (j, g) is g + 4 v (not 4 g + v).
// Row i of m-block mb is therefore (x tap a = mb + 4 (i & 1), rhs
// r8 = 4 ((i >> 1) & 1) + (i >> 2)), so that a lane's four results are four
// consecutive right-hand sides of one x tap (lane group g: a = mb + 4 (g & 1),
// r8 = 4 (g >> 1) + v) and the four x taps of a lane's A operands are four
// consecutive doubles of the record.
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
constexpr int RHW = 8;      // right-hand sides per wavefront in the FP64 contractions
__device__ inline int row_rhs64(int i) { return 4 * ((i >> 1) & 1) + (i >> 2); }
constexpr int REC64 = 24;   // doubles per FP64 point record: x, y and z taps

// CHB records as stored (24 doubles each, 6 KB): 1 KB slot j, lane l moves bytes
// 1024 j + 16 l of the chunk (one 16-byte piece of record (1024 j + 16 l) / 192).
// Wavefront `w` of the block moves slots w, w + 2, ...
__device__ inline void stage_records64(double* lrec, const double* __restrict__ wts, int64_t base, int cstart,
                                       int count, int lane, int w) {
    const int last = count - 1 - cstart;
#pragma unroll
    for (int j2 = 0; j2 < CHB * REC64 * 8 / 2048; ++j2) {
        const int j = 2 * j2 + w;
        const int o = j * 1024 + lane * 16;
        dma16(wts + (base + cstart + min(o / (REC64 * 8), last)) * REC64 + (o % (REC64 * 8)) / 8, lrec + j * 128);
    }
}

// CHB records with the z taps repeated (32 doubles each, 8 KB), so that any 8
// cyclically consecutive z taps are 8 consecutive doubles: 4 records per slot.
// Records for the FP64 gather: 16 pieces of 16 bytes (the x and y taps, then the
// z taps twice, so that 8 consecutive z taps can be read from any start) and a
// 17th of padding, so that the records of consecutive points start 68 words
// apart: the 16 points a step reads at the same offset fall on different LDS
// banks (with records 256 bytes apart they all fell on the same ones). Slot s of
// a chunk holds piece s % 17 of record s / 17; the 544 slots of a chunk go out
// as 8 1 KB direct loads and a half one, split between the two wavefronts.
constexpr int kRecSlots64 = 17;
__device__ inline void stage_records64_ring(double* lrec, const double* __restrict__ wts, int64_t base, int cstart,
                                            int count, int lane, int w) {
    const int last = count - 1 - cstart;
    constexpr int NS = CHB * kRecSlots64;  // 16-byte slots of a chunk
#pragma unroll
    for (int j2 = 0; j2 < (NS + 127) / 128; ++j2) {
        const int j = 2 * j2 + w;
        const int sl = j * 64 + lane;
        if (j * 64 < NS && sl < NS) {
            const int rec = sl / kRecSlots64, piece = sl % kRecSlots64;
            const int e = piece < 12 ? 2 * piece : (piece < 16 ? 2 * piece - 8 : 0);
            dma16(wts + (base + cstart + min(rec, last)) * REC64 + e, lrec + j * 128);
        }
    }
}

// The next work item of a two-wavefront block (taken by its first thread from
// the queue shared by the resident blocks; the trailing barrier keeps the slot
// from being overwritten before both wavefronts have read it).
__device__ inline int next_item(int32_t* queue, int* slot) {
    if (threadIdx.x == 0) *slot = atomicAdd(queue, 1);
    __syncthreads();
    const int it = *slot;
    __syncthreads();
    return it;
}

// This wavefront's 8 right-hand sides of two value rows (16 rows per slot,
// 64 bytes each: four lanes per row).
__device__ inline void stage_values64(double* lval, const double* __restrict__ xt, const int32_t (&pr)[2], int half,
                                      int lane) {
#pragma unroll
    for (int j = 0; j < 2; ++j) dma16(xt + int64_t(pr[j]) * RB + RHW * half + (lane % 4) * 2, lval + j * 128);
}

__device__ inline void lds_spread_operands64(uint32_t ax, uint32_t ay, uint32_t az, uint32_t av, d2& wx01, d2& wx23,
                                             d2& wy01, d2& wy23, double& wz, double& v) {
    asm volatile(
        "ds_read_b128 %0, %6\n\t"
        "ds_read_b128 %1, %6 offset:16\n\t"
        "ds_read_b128 %2, %7\n\t"
        "ds_read_b128 %3, %7 offset:16\n\t"
        "ds_read_b64 %4, %8\n\t"
        "ds_read_b64 %5, %9\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(wx01), "=&v"(wx23), "=&v"(wy01), "=&v"(wy23), "=&v"(wz), "=&v"(v)
        : "v"(ax), "v"(ay), "v"(az), "v"(av)
        : "memory");
}

__device__ inline void lds_gather_operands64(uint32_t ax, uint32_t ay, uint32_t az, d2& wx01, d2& wx23, double& wy0,
                                             double& wy1, double (&wz)[8]) {
    asm volatile(
        "ds_read_b128 %0, %12\n\t"
        "ds_read_b128 %1, %12 offset:16\n\t"
        "ds_read_b64 %2, %13\n\t"
        "ds_read_b64 %3, %13 offset:32\n\t"
        "ds_read_b64 %4, %14\n\t"
        "ds_read_b64 %5, %14 offset:8\n\t"
        "ds_read_b64 %6, %14 offset:16\n\t"
        "ds_read_b64 %7, %14 offset:24\n\t"
        "ds_read_b64 %8, %14 offset:32\n\t"
        "ds_read_b64 %9, %14 offset:40\n\t"
        "ds_read_b64 %10, %14 offset:48\n\t"
        "ds_read_b64 %11, %14 offset:56\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(wx01), "=&v"(wx23), "=&v"(wy0), "=&v"(wy1), "=&v"(wz[0]), "=&v"(wz[1]), "=&v"(wz[2]), "=&v"(wz[3]),
          "=&v"(wz[4]), "=&v"(wz[5]), "=&v"(wz[6]), "=&v"(wz[7])
        : "v"(ax), "v"(ay), "v"(az)
        : "memory");
}

__device__ inline void lds_store_d2(uint32_t addr, d2 v) {
    asm volatile("ds_write_b128 %0, %1" : : "v"(addr), "v"(v) : "memory");
}

__device__ inline d2 lds_load_d2(uint32_t addr) {
    d2 v;
    asm volatile("ds_read_b128 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=&v"(v) : "v"(addr) : "memory");
    return v;
}

// Spread, FP64. Accumulator tile (mb, nb) of 16 x 16: rows as above, columns
// n = lr -> (y tap b = nb + 4 (lr >> 3), physical z column lr & 7); the lane
// (lr, lk) holds x tap mb + 4 (lk & 1) and right-hand sides 4 (lk >> 1) .. + 3
// of its half, in column lr. A step takes 4 points.
__global__ __launch_bounds__(128, 2) void k_spread_mfma64(const int32_t* __restrict__ wave_items, int32_t nwork,
                                                         int32_t* __restrict__ queue,
                                                         const Segment* __restrict__ segs,
                                                         const int32_t* __restrict__ lstart,
                                                         const int32_t* __restrict__ lstart_off,
                                                         const WinDev* __restrict__ wins,
                                                         const uint8_t* __restrict__ alone,
                                                         const double* __restrict__ wts,
                                                         const int32_t* __restrict__ perm,
                                                         const double* __restrict__ xt, int64_t N,
                                                         double* __restrict__ slab, double* __restrict__ tgt) {
    constexpr int STEP = CHB - 4;
    __shared__ __align__(16) double srec[2][CHB * REC64];
    __shared__ __align__(16) double svals[2][2][CHB * RHW];
    __shared__ __align__(16) double stgs[2][64 * RHW];
    __shared__ int slot;
    const int lane = threadIdx.x & 63;
    const int half = threadIdx.x >> 6;  // the wavefront's half of the right-hand sides
    double(&sval)[2][CHB * RHW] = svals[half];
    double* const stg = stgs[half];
    for (;;) {
        const int it = next_item(queue, &slot);
        if (it >= nwork) break;
        const int sid = wave_items[it];
        const Segment sg = segs[sid];
        const WinDev& wd = wins[sg.win];
        const int lr = lane & 15, lk = lane >> 4;
        const int64_t base = int64_t(sg.win) * N + sg.start;
        const int32_t* ls = lstart + lstart_off[sid];
        const bool direct = alone[sid] != 0;
        const int cx = sg.col / wd.nb[1], cy = sg.col % wd.nb[1];
        const int E1 = wd.E[1], E2 = wd.E[2];
        // output addressing as in k_spread_mfma
        const int64_t SA = direct ? int64_t(64 * E1 + 8) * E2 : 8;
        const int64_t SB = direct ? int64_t(65) * E2 : 1;
        const int64_t U0 = direct ? wd.tgt_off + (int64_t(cx) * E1 + cy) * 64 * E2 : sg.off - int64_t(sg.z0) * 64;
        const int64_t UL = direct ? 1 : 64;
        double* const outp = direct ? tgt : slab;
        d4 acc[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
        // Write z cell `layer` of this half and clear it: rows [8 a + b][8 rhs]
        // through LDS, then four lanes per 64-byte half row.
        const uint32_t stg0 = lds_addr(&stg[0]);
        auto flush = [&](int layer) __attribute__((always_inline)) {
            if ((lr & 7) == (layer & 7)) {
#pragma unroll
                for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb) {
                        const int ab = (mb + 4 * (lk & 1)) * 8 + nb + 4 * (lr >> 3);
                        const uint32_t ad = stg0 + uint32_t(ab * RHW + 4 * (lk >> 1)) * 8;
                        const d4 a = acc[mb * 4 + nb];
                        lds_store_d2(ad, d2{a[0], a[1]});
                        lds_store_d2(ad + 16, d2{a[2], a[3]});
                        acc[mb * 4 + nb] = d4{0.0, 0.0, 0.0, 0.0};
                    }
            }
            lds_wait();
            __syncthreads();
            double* const row = outp + (U0 + int64_t(layer) * UL) * RB + RHW * half + 2 * (lane & 3);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ab = 16 * j + (lane >> 2);
                const d2 v = lds_load_d2(stg0 + uint32_t(ab * RHW + 2 * (lane & 3)) * 8);
                *reinterpret_cast<d2*>(row + ((ab >> 3) * SA + (ab & 7) * SB) * RB) = v;
            }
        };
        const uint32_t rec0 = lds_addr(&srec[0][0]), val0 = lds_addr(&sval[0][0]);
        constexpr uint32_t RECB = CHB * REC64 * 8, VALB = CHB * RHW * 8;  // bytes per buffer
        int cc = -1;
        int32_t prow[2];
        stage_records64(srec[0], wts, base, 0, sg.count, lane, half);
        value_rows(perm, base, 0, sg.count, lane, prow);
        stage_values64(sval[0], xt, prow, half, lane);
        if (STEP < sg.count) value_rows(perm, base, STEP, sg.count, lane, prow);
        for (int z = sg.z0; z <= sg.z1; ++z) {
            const int p = ls[z - sg.z0], q = ls[z - sg.z0 + 1];
            for (int k = p; k < q; k += 4) {
                const int c = k / STEP;
                if (c > cc) {  // chunk c has landed (and earlier stores have drained); prefetch c + 1
                    wait_vmem_b();
                    __syncthreads();
                    cc = c;
                    if ((c + 1) * STEP < sg.count) {
                        stage_records64(srec[(c + 1) & 1], wts, base, (c + 1) * STEP, sg.count, lane, half);
                        stage_values64(sval[(c + 1) & 1], xt, prow, half, lane);
                        if ((c + 2) * STEP < sg.count) value_rows(perm, base, (c + 2) * STEP, sg.count, lane, prow);
                    }
                }
                const int pt = k + lk;
                const uint32_t slot = uint32_t(pt - c * STEP);
                const uint32_t rb = rec0 + uint32_t(c & 1) * RECB + slot * (REC64 * 8);
                d2 wx01, wx23, wy01, wy23;
                double wz, v;
                lds_spread_operands64(rb + 32 * uint32_t(lr & 1), rb + 64 + 32 * uint32_t(lr >> 3),
                                      rb + 128 + 8 * uint32_t((lr - z) & 7),
                                      val0 + uint32_t(c & 1) * VALB + (slot * RHW + row_rhs64(lr)) * 8, wx01, wx23,
                                      wy01, wy23, wz, v);
                v = pt < q ? v : 0.0;
                const double av[4] = {v * wx01[0], v * wx01[1], v * wx23[0], v * wx23[1]};
                const double bv[4] = {wy01[0] * wz, wy01[1] * wz, wy23[0] * wz, wy23[1] * wz};
#pragma unroll
                for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb)
                        acc[mb * 4 + nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mb], bv[nb], acc[mb * 4 + nb], 0, 0, 0);
            }
            flush(z);
        }
        for (int j = 1; j < 8; ++j) flush(sg.z1 + j);
    }
}

// Gather, FP64: S[(a, r)][p] = sum_K H[(a, r)][K] B[K][p] over the 64 taps, in
// 16 k-steps ks of 4: k-index lk of step ks is tap (y tap b = 4 (ks >> 3) + lk,
// ring column c = ks & 7), so a lane holds one tap of each ring column per
// y-tap group and refilling column c after a layer touches H[.][c] and
// H[.][c + 8] in every lane. D[mb] holds, in lane (point lr, lk), the rows
// (x tap mb + 4 (lk & 1), rhs 4 (lk >> 1) .. + 3); f sums the x taps of
// a < 4 in the lanes with even lk, adds those of a >= 4 from lane + 16, and
// stores.
__global__ __launch_bounds__(128, 2) void k_gather_mfma64(const int32_t* __restrict__ wave_items, int32_t nwork,
                                                         int32_t* __restrict__ queue,
                                                         const Segment* __restrict__ segs,
                                                         const int32_t* __restrict__ lstart,
                                                         const int32_t* __restrict__ lstart_off,
                                                         const WinDev* __restrict__ wins,
                                                         const double* __restrict__ wts,
                                                         const double* __restrict__ h, int64_t N,
                                                         double* __restrict__ fs) {
    constexpr int STEP = CHB - 16;
    constexpr int RPD = 2 * kRecSlots64;  // doubles per staged record (z taps repeated, one padding piece)
    __shared__ __align__(16) double srec[2][CHB * RPD];
    __shared__ int slot;
    const int lane = threadIdx.x & 63;
    const int half = threadIdx.x >> 6;  // the wavefront's half of the right-hand sides
    for (;;) {
        const int it = next_item(queue, &slot);
        if (it >= nwork) break;
        const int sid = wave_items[it];
        const Segment sg = segs[sid];
        const WinDev& wd = wins[sg.win];
        const int lr = lane & 15, lk = lane >> 4;
        const int64_t base = int64_t(sg.win) * N + sg.start;
        const int32_t* ls = lstart + lstart_off[sid];
        const int cx = sg.col / wd.nb[1], cy = sg.col % wd.nb[1];
        const int Ey = wd.E[1], Ez = wd.E[2];
        // h[x][z][y][r]: rows of this lane are x = cx + mb + 4 (lr & 1), rhs 8 half + row_rhs64(lr)
        const double* hp = h + (wd.grid_off + int64_t(cx + 4 * (lr & 1)) * Ez * Ey + cy + lk) * RB + RHW * half +
                           row_rhs64(lr);
        double H[4][16];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const int layer = sg.z0 + (((ks & 7) - sg.z0) & 7);
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) H[mb][ks] = hp[((int64_t(mb) * Ez + layer) * Ey + 4 * (ks >> 3)) * RB];
        }
        double pre[4][2];
        if (sg.z0 < sg.z1) {
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                for (int k2 = 0; k2 < 2; ++k2) pre[mb][k2] = hp[((int64_t(mb) * Ez + sg.z0 + 8) * Ey + 4 * k2) * RB];
        }
        const uint32_t rec0 = lds_addr(&srec[0][0]);
        constexpr uint32_t RECB = CHB * RPD * 8;
        int cc = -1;
        stage_records64_ring(srec[0], wts, base, 0, sg.count, lane, half);
        for (int z = sg.z0; z <= sg.z1; ++z) {
            const int p = ls[z - sg.z0], q = ls[z - sg.z0 + 1];
            for (int k = p; k < q; k += 16) {
                const int c = k / STEP;
                if (c > cc) {
                    wait_vmem_b();
                    __syncthreads();
                    cc = c;
                    if ((c + 1) * STEP < sg.count)
                        stage_records64_ring(srec[(c + 1) & 1], wts, base, (c + 1) * STEP, sg.count, lane, half);
                }
                const int pt = k + lr;
                const uint32_t rb = rec0 + uint32_t(c & 1) * RECB + uint32_t(pt - c * STEP) * (RPD * 8);
                d2 wx01, wx23;
                double wy0, wy1, wz[8];  // wz[c]: z tap of ring column c, (c - z) & 7
                lds_gather_operands64(rb + 32 * uint32_t(lk & 1), rb + 64 + 8 * uint32_t(lk),
                                      rb + 128 + 8 * uint32_t((-z) & 7), wx01, wx23, wy0, wy1, wz);
                double B[16];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    B[j] = wy0 * wz[j];
                    B[8 + j] = wy1 * wz[j];
                }
                d4 D[4];
#pragma unroll
                for (int mb = 0; mb < 4; ++mb) D[mb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < 16; ++ks)
#pragma unroll
                    for (int mb = 0; mb < 4; ++mb) D[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(H[mb][ks], B[ks], D[mb], 0, 0, 0);
                d4 f = wx01[0] * D[0];
                f += wx01[1] * D[1];
                f += wx23[0] * D[2];
                f += wx23[1] * D[3];
                d4 o;
#pragma unroll
                for (int i = 0; i < 4; ++i) o[i] = __shfl_xor(f[i], 16);
                if ((lk & 1) == 0 && pt < q)
                    *reinterpret_cast<d4*>(fs + (base + pt) * RB + RHW * half + 4 * (lk >> 1)) = f + o;
            }
            if (z < sg.z1) {  // column z mod 8 takes layer z + 8; load layer z + 9 for the next column
                switch (z & 7) {
#define ANV_REFILL64(J)                                  \
    case J:                                              \
        _Pragma("unroll") for (int mb = 0; mb < 4; ++mb) { \
            H[mb][J] = pre[mb][0];                       \
            H[mb][J + 8] = pre[mb][1];                   \
        }                                                \
        break;
                    ANV_REFILL64(0) ANV_REFILL64(1) ANV_REFILL64(2) ANV_REFILL64(3)
                    ANV_REFILL64(4) ANV_REFILL64(5) ANV_REFILL64(6) ANV_REFILL64(7)
#undef ANV_REFILL64
                }
                if (z + 1 < sg.z1) {
#pragma unroll
                    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                        for (int k2 = 0; k2 < 2; ++k2)
                            pre[mb][k2] = hp[((int64_t(mb) * Ez + z + 9) * Ey + 4 * k2) * RB];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- 1 and 2 features: one lane per (item, rhs)
template <int W, int WY, class T>
__global__ __launch_bounds__(64) void k_spread_lane_b(const int32_t* __restrict__ items, int nitems,
                                                      const Segment* __restrict__ segs,
                                                      const int32_t* __restrict__ zq,
                                                      const T* __restrict__ wts,
                                                      const int32_t* __restrict__ perm,
                                                      const T* __restrict__ xt, int64_t N,
                                                      T* __restrict__ slab) {
    const int64_t t = blockIdx.x * int64_t(64) + threadIdx.x;
    if (t >= int64_t(nitems) * RB) return;
    const int sid = items[t / RB];
    const int r = int(t % RB);
    if (sid < 0) return;
    const Segment sg = segs[sid];
    const int64_t base = int64_t(sg.win) * N + sg.start;
    constexpr int REC = rec_stride(W, int(sizeof(T)));
    T acc[WY][W];
#pragma unroll
    for (int b = 0; b < WY; ++b)
#pragma unroll
        for (int c = 0; c < W; ++c) acc[b][c] = T(0);
    int zr = sg.z0;
    for (int k = 0; k < sg.count; ++k) {
        const int64_t gi = base + k;
        const int zj = zq[gi];
        while (zr < zj) {
#pragma unroll
            for (int b = 0; b < WY; ++b) slab[(sg.off + int64_t(zr - sg.z0) * WY + b) * RB + r] = acc[b][0];
#pragma unroll
            for (int b = 0; b < WY; ++b) {
#pragma unroll
                for (int c = 0; c < W - 1; ++c) acc[b][c] = acc[b][c + 1];
                acc[b][W - 1] = T(0);
            }
            ++zr;
        }
        const T* w = wts + gi * REC;
        const T v = xt[int64_t(perm[gi]) * RB + r];
#pragma unroll
        for (int b = 0; b < WY; ++b) {
            const T cb = v * w[W + b];
#pragma unroll
            for (int c = 0; c < W; ++c) acc[b][c] += cb * w[2 * W + c];
        }
    }
#pragma unroll
    for (int c = 0; c < W; ++c)
#pragma unroll
        for (int b = 0; b < WY; ++b) slab[(sg.off + int64_t(zr - sg.z0 + c) * WY + b) * RB + r] = acc[b][c];
}

template <int W, int WY, class T>
__global__ __launch_bounds__(64) void k_gather_lane_b(const int32_t* __restrict__ items, int nitems,
                                                      const Segment* __restrict__ segs,
                                                      const WinDev* __restrict__ wins,
                                                      const int32_t* __restrict__ zq,
                                                      const T* __restrict__ wts,
                                                      const T* __restrict__ h, int64_t N,
                                                      T* __restrict__ fs) {
    const int64_t t = blockIdx.x * int64_t(64) + threadIdx.x;
    if (t >= int64_t(nitems) * RB) return;
    const int sid = items[t / RB];
    const int r = int(t % RB);
    if (sid < 0) return;
    const Segment sg = segs[sid];
    const WinDev& wd = wins[sg.win];
    const int cx = sg.col / wd.nb[1], cy = sg.col % wd.nb[1];
    const int Ey = wd.E[1];
    const T* hp = h + (wd.grid_off + int64_t(cx) * wd.E[2] * Ey + cy) * RB + r;
    const int64_t base = int64_t(sg.win) * N + sg.start;
    constexpr int REC = rec_stride(W, int(sizeof(T)));
    T hr[WY][W];
    int zr = sg.z0;
#pragma unroll
    for (int c = 0; c < W; ++c)
#pragma unroll
        for (int b = 0; b < WY; ++b) hr[b][c] = hp[(int64_t(zr + c) * Ey + b) * RB];
    for (int k = 0; k < sg.count; ++k) {
        const int64_t gi = base + k;
        const int zj = zq[gi];
        while (zr < zj) {
#pragma unroll
            for (int b = 0; b < WY; ++b) {
#pragma unroll
                for (int c = 0; c < W - 1; ++c) hr[b][c] = hr[b][c + 1];
                hr[b][W - 1] = hp[(int64_t(zr + W) * Ey + b) * RB];
            }
            ++zr;
        }
        const T* w = wts + gi * REC;
        T sy = T(0);
#pragma unroll
        for (int b = 0; b < WY; ++b) {
            T s = T(0);
#pragma unroll
            for (int c = 0; c < W; ++c) s += w[2 * W + c] * hr[b][c];
            sy += w[W + b] * s;
        }
        fs[gi * RB + r] = sy;
    }
}

// ---------------------------------------------------------------- fold and grid step, 16 rhs innermost
template <class T>
__global__ __launch_bounds__(256) void k_fold_cols_b(const WinDev* __restrict__ wins, int32_t P, int64_t nlist,
                                                     const int64_t* __restrict__ flist, const int2* __restrict__ fold,
                                                     const int64_t* __restrict__ sbase, const T* __restrict__ slab,
                                                     T* __restrict__ tgt) {
    __shared__ double red[256][4];
    const int64_t fi = blockIdx.x;
    if (fi >= nlist) return;
    const int64_t f = flist[fi];
    int l = 0;
    while (l + 1 < P && wins[l + 1].fold_off <= f) ++l;
    const WinDev& wd = wins[l];
    // thread = (part, footprint position, rhs quad): the items covering the cell
    // are dealt to the parts in turn, and the parts' sums are added in part order
    const int lanes = wd.lanes, parts = 64 / lanes;
    const int t = threadIdx.x, q4 = t % 4, rest = t / 4;
    const int pos = rest % lanes, part = rest / lanes;
    const int64_t fl = f - wd.fold_off;
    const int L = int(fl % wd.E[2]);
    const int64_t col = fl / wd.E[2];
    const int cx = int(col / wd.nb[1]), cy = int(col % wd.nb[1]);
    const int a = pos / wd.Wslot[1], b = pos % wd.Wslot[1];
    const int2 rr = fold[f];
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    if (part < parts) {
        auto at = [&](int s) __attribute__((always_inline)) {
            return *reinterpret_cast<const v4<T>*>(slab + (sbase[s] + int64_t(L) * lanes + pos) * RB + 4 * q4);
        };
        auto add = [&](const v4<T>& v) __attribute__((always_inline)) {
            s0 += v[0];
            s1 += v[1];
            s2 += v[2];
            s3 += v[3];
        };
        int s = rr.x + part;
        // four items' loads in flight at a time, added in item order
        for (; s + 3 * parts < rr.y; s += 4 * parts) {
            const v4<T> v0 = at(s), v1 = at(s + parts), v2 = at(s + 2 * parts), v3 = at(s + 3 * parts);
            add(v0);
            add(v1);
            add(v2);
            add(v3);
        }
        for (; s < rr.y; s += parts) add(at(s));
    }
    red[t][0] = s0;
    red[t][1] = s1;
    red[t][2] = s2;
    red[t][3] = s3;
    __syncthreads();
    if (part != 0 || rest >= lanes) return;
    double o[4] = {0, 0, 0, 0};
    for (int q = 0; q < parts; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] += red[(q * lanes + pos) * 4 + q4][i];
    const int64_t tt = ((int64_t(cx + a) * wd.E[1] + (cy + b)) * lanes + pos) * wd.E[2] + L;
    *reinterpret_cast<v4<T>*>(tgt + (wd.tgt_off + tt) * RB + 4 * q4) = v4<T>{T(o[0]), T(o[1]), T(o[2]), T(o[3])};
}

// Blocks are dealt to the 8 XCDs in turn (block i to XCD i mod 8). The nrs
// right-hand-side slices of one (slice, window) group go to one XCD back to
// back, so that the slices after the first find the group's 64-byte rows (all
// 16 right-hand sides) in that XCD's L2. Group g = window * ne + slice; blocks
// past the last group return.
__device__ inline bool xcd_group(int nrs, int ne, int ngroups, int& slice, int& l, int& rs) {
    const int b = int(blockIdx.x), k = b >> 3;
    rs = k % nrs;
    const int g = (k / nrs) * 8 + (b & 7);
    l = g / ne;
    slice = g % ne;
    return g < ngroups;
}

// fold step B + y and z passes; block per (x slice, window, slice of the rhs)
// FP64: blocks of 512 threads, whose 256 registers per lane hold the fold's 64
// loads in flight without spilling (1024-thread blocks have 128)
template <class T>
constexpr int fold_conv_threads() { return sizeof(T) == 8 ? 512 : 1024; }
template <int W, class T>
__global__ __launch_bounds__(fold_conv_threads<T>()) void k_fold_conv_yz_b(const WinDev* __restrict__ wins,
                                                         const double* __restrict__ tmat,
                                                         const int2* __restrict__ crange,
                                                         const T* __restrict__ tgt, T* __restrict__ g1,
                                                         int RH, int ne, int P) {
    extern __shared__ __align__(16) unsigned char sm_raw[];
    T* const smf = reinterpret_cast<T*>(sm_raw);
    int x, l, rs;
    if (!xcd_group(RB / RH, ne, ne * P, x, l, rs)) return;
    const WinDev& wd = wins[l];
    const int r0 = rs * RH;
    if (x >= wd.E[0]) return;
    const int Ey = wd.E[1], Ez = wd.E[2];
    const int Eyp = (Ey + 3) & ~3, Ezp = (Ez + 3) & ~3;
    const int S = Ey * Ez;
    // Toeplitz matrices transposed, rows padded to a multiple of 4 with zeros:
    // tyT[k][y] = Ty[y][k], so that 4 consecutive outputs read their 4
    // coefficients of tap k in one 16-byte access
    T* tyT = smf;
    T* tzT = tyT + Ey * Eyp;
    T* s0 = tzT + Ez * Ezp;  // [y][z][RH]
    T* s1 = s0 + S * RH;
    for (int e = threadIdx.x; e < Ey * Eyp; e += blockDim.x) {
        const int k = e / Eyp, y = e % Eyp;
        tyT[e] = y < Ey ? T(tmat[wd.t_off[1] + y * Ey + k]) : T(0);
    }
    for (int e = threadIdx.x; e < Ez * Ezp; e += blockDim.x) {
        const int k = e / Ezp, z = e % Ezp;
        tzT[e] = z < Ez ? T(tmat[wd.t_off[2] + z * Ez + k]) : T(0);
    }
    __shared__ int2 rng[W][65];
    const int wx = wd.Wslot[0], wy = wd.Wslot[1], nby = wd.nb[1];
    for (int e = threadIdx.x; e < W * nby; e += blockDim.x) {
        const int a = e / nby, cyy = e % nby, cxx = x - a;
        rng[a][cyy] = (a < wx && cxx >= 0 && cxx < wd.nb[0]) ? crange[wd.col_off + int64_t(cxx) * nby + cyy]
                                                            : make_int2(1, 0);
    }
    __syncthreads();
    // fold step B: s0[y][z][r] = sum over the footprint positions (a, b) whose
    // column holds points at layers reaching z, in (a, b) order
    for (int e = threadIdx.x; e < S * RH; e += blockDim.x) {
        const int cell = e / RH, r = e % RH;
        const int y = cell / Ez, zz = cell % Ez;
        const T* tl = tgt + (wd.tgt_off + (int64_t(x) * Ey + y) * wd.lanes * Ez + zz) * RB + r0 + r;
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < W; ++a)
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const int cyy = y - b;
                const int2 rr = (b < wy && cyy >= 0 && cyy < nby) ? rng[a][cyy] : make_int2(1, 0);
                // the target holds no valid value where the position's column has
                // no points reaching layer z; every lane loads (a valid address) so
                // that all 64 loads are in flight at once, and the select drops it
                const bool ok = zz >= rr.x && zz <= rr.y;
                const T v = tl[ok ? int64_t(a * wy + b) * Ez * RB : 0];
                acc += ok ? v : T(0);
            }
        s0[e] = acc;
    }
    __syncthreads();
    // y pass, s1[y][z][r] = sum_k Ty[y][k] s0[k][z][r] (k ascending); a thread
    // makes y = y0 .. y0 + 3 from one read of s0 per tap
    for (int e = threadIdx.x; e < (Eyp / 4) * Ez * RH; e += blockDim.x) {
        const int r = e % RH, zz = (e / RH) % Ez, y0 = 4 * (e / (RH * Ez));
        T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
        for (int k = 0; k < Ey; ++k) {
            const T v = s0[(k * Ez + zz) * RH + r];
            const v4<T> t = *reinterpret_cast<const v4<T>*>(tyT + k * Eyp + y0);
            a0 += t[0] * v;
            a1 += t[1] * v;
            a2 += t[2] * v;
            a3 += t[3] * v;
        }
        const T av[4] = {a0, a1, a2, a3};
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (y0 + i < Ey) s1[((y0 + i) * Ez + zz) * RH + r] = av[i];
    }
    __syncthreads();
    // z pass, g1[x][y][z][r] = sum_k Tz[z][k] s1[y][k][r]; z = z0 .. z0 + 3 per thread
    T* out = g1 + (wd.grid_off + int64_t(x) * S) * RB + r0;
    for (int e = threadIdx.x; e < Ey * (Ezp / 4) * RH; e += blockDim.x) {
        const int r = e % RH, z0 = 4 * ((e / RH) % (Ezp / 4)), y = e / (RH * (Ezp / 4));
        T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
        for (int k = 0; k < Ez; ++k) {
            const T v = s1[(y * Ez + k) * RH + r];
            const v4<T> t = *reinterpret_cast<const v4<T>*>(tzT + k * Ezp + z0);
            a0 += t[0] * v;
            a1 += t[1] * v;
            a2 += t[2] * v;
            a3 += t[3] * v;
        }
        const T av[4] = {a0, a1, a2, a3};
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (z0 + i < Ez) out[int64_t(y * Ez + z0 + i) * RB + r] = av[i];
    }
}

// x pass; block per (y slice, window, rhs half); output h[x][z][y][rhs]
template <class T>
__global__ __launch_bounds__(1024) void k_conv_x_b(const WinDev* __restrict__ wins, const double* __restrict__ tmat,
                                                   const T* __restrict__ g1, T* __restrict__ h, int RH, int ne,
                                                   int P) {
    extern __shared__ __align__(16) unsigned char sm_raw[];
    T* const smf = reinterpret_cast<T*>(sm_raw);
    int y, l, rs;
    if (!xcd_group(RB / RH, ne, ne * P, y, l, rs)) return;
    const WinDev& wd = wins[l];
    const int r0 = rs * RH;
    if (y >= wd.E[1]) return;
    const int Ex = wd.E[0], Ey = wd.E[1], Ez = wd.E[2];
    const int Exp = (Ex + 3) & ~3;
    T* txT = smf;                // txT[k][x] = Tx[x][k], rows padded to Exp
    T* sl = smf + Ex * Exp;      // [x][z][RH]
    for (int e = threadIdx.x; e < Ex * Exp; e += blockDim.x) {
        const int k = e / Exp, xx = e % Exp;
        txT[e] = xx < Ex ? T(tmat[wd.t_off[0] + xx * Ex + k]) : T(0);
    }
    for (int e = threadIdx.x; e < Ex * Ez * RH; e += blockDim.x) {
        const int xz = e / RH, r = e % RH;
        const int xx = xz / Ez, zz = xz % Ez;
        sl[e] = g1[(wd.grid_off + (int64_t(xx) * Ey + y) * Ez + zz) * RB + r0 + r];
    }
    __syncthreads();
    // h[x][z][y][r] = sum_k Tx[x][k] g1[k][y][z][r] (k ascending); x = x0 .. x0 + 3 per thread
    for (int e = threadIdx.x; e < (Exp / 4) * Ez * RH; e += blockDim.x) {
        const int r = e % RH, zz = (e / RH) % Ez, x0 = 4 * (e / (RH * Ez));
        T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
        for (int k = 0; k < Ex; ++k) {
            const T v = sl[(k * Ez + zz) * RH + r];
            const v4<T> t = *reinterpret_cast<const v4<T>*>(txT + k * Exp + x0);
            a0 += t[0] * v;
            a1 += t[1] * v;
            a2 += t[2] * v;
            a3 += t[3] * v;
        }
        const T av[4] = {a0, a1, a2, a3};
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (x0 + i < Ex) h[(wd.grid_off + (int64_t(x0 + i) * Ez + zz) * Ey + y) * RB + r0 + r] = av[i];
    }
}

// y_r[i] = sum_l eta_l f_l(i, r), windows in order, FP64; 64 points per
// block, a thread takes 4 right-hand sides of one point; the windows' rows are
// loaded 8 at a time, all in flight together; transposed through LDS for
// coalesced stores
constexpr int kWsChunk = 8;
template <class T>
__global__ __launch_bounds__(256) void k_window_sum_b(const T* __restrict__ fs, const int32_t* __restrict__ pos,
                                                      const WinDev* __restrict__ wins, int32_t P, int64_t N, int R,
                                                      const ColPtrs cols) {
    __shared__ double s[RB][65];
    const int64_t i0 = int64_t(blockIdx.x) * 64;
    const int i = threadIdx.x >> 2, q = threadIdx.x & 3;
    const int64_t gi = i0 + i;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (gi < N) {
        for (int l0 = 0; l0 < P; l0 += kWsChunk) {
            int32_t pp[kWsChunk];
#pragma unroll
            for (int j = 0; j < kWsChunk; ++j) pp[j] = l0 + j < P ? pos[int64_t(l0 + j) * N + gi] : 0;
            v4<T> v[kWsChunk];
#pragma unroll
            for (int j = 0; j < kWsChunk; ++j)
                v[j] = l0 + j < P ? *reinterpret_cast<const v4<T>*>(fs + (int64_t(l0 + j) * N + pp[j]) * RB + 4 * q)
                                  : v4<T>{T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int j = 0; j < kWsChunk; ++j) {
                if (l0 + j < P) {
                    const double eta = wins[l0 + j].eta;
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c] += eta * double(v[j][c]);
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) s[4 * q + c][i] = acc[c];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = j * 256 + threadIdx.x;
        const int r = e / 64, i = e % 64;  // r is uniform across a wavefront
        if (r < R && i0 + i < N) cols.y[r][i0 + i] = s[r][i];
    }
}

}  // namespace

bool batched_supported(const Plan& pl) {
    return (pl.precision == ANOVA_PREC_MIXED || pl.precision == ANOVA_PREC_FP64) && pl.W == 8;
}

namespace {
template <class T>
T* buf_as(DevBuf<double>& b) {
    return reinterpret_cast<T*>(b.p);
}
// a batched buffer of n elements of elem bytes (storage in whole doubles)
void alloc_elems(DevBuf<double>& b, size_t n, size_t elem) { b.alloc((n * elem + 7) / 8); }
}  // namespace

void release_batched_buffers(Plan& pl) {
    for (DevBuf<double>* b : {&pl.xtb, &pl.fsb, &pl.slabb, &pl.tgtb, &pl.g1b, &pl.hb}) b->release();
    pl.b_items.release();
    pl.b_queue.release();
    pl.b_ready = false;
}

void ensure_batched_buffers(Plan& pl) {
    if (pl.b_ready) return;
    const bool f64 = pl.precision == ANOVA_PREC_FP64;
    const size_t elem = f64 ? sizeof(double) : sizeof(float);
    alloc_elems(pl.xtb, size_t(pl.N) * RB, elem);
    alloc_elems(pl.fsb, size_t(pl.N) * pl.P * RB, elem);
    alloc_elems(pl.slabb, size_t(pl.slab_total) * RB + RB, elem);
    alloc_elems(pl.tgtb, size_t(pl.tgt_total) * RB, elem);
    alloc_elems(pl.g1b, size_t(pl.grid_total) * RB, elem);
    alloc_elems(pl.hb, size_t(pl.grid_total) * RB, elem);
    // items of 1- and 2-feature windows as flat lists (lane kernels take (item, rhs) per lane)
    std::vector<int32_t> it2, it1;
    for (size_t i = 0; i < pl.segs_h.size(); ++i) {
        int l = pl.segs_h[i].win;
        int dw = 0;
        for (int s2 = 0; s2 < 3; ++s2) dw += pl.slot_feat[l][s2] >= 0;
        if (dw == 2) it2.push_back(int32_t(i));
        if (dw == 1) it1.push_back(int32_t(i));
    }
    pl.nb_items2 = int32_t(it2.size());
    pl.nb_items1 = int32_t(it1.size());
    it2.insert(it2.end(), it1.begin(), it1.end());
    if (it2.empty()) it2.push_back(-1);
    pl.b_items.alloc(it2.size());
    ANV_HIP(hipMemcpy(pl.b_items.p, it2.data(), it2.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    // persistent grids of the matrix-core kernels: as many wavefronts as fit at
    // once (the FP64 kernels take a work item per half of the right-hand sides)
    pl.b_queue.alloc(2);
    {
        int dev = 0, ncu = 0, bs = 0, bg = 0;
        ANV_HIP(hipGetDevice(&dev));
        ANV_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        if (f64) {
            ANV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&bs, k_spread_mfma64, 128, 0));
            ANV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&bg, k_gather_mfma64, 128, 0));
        } else {
            ANV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&bs, k_spread_mfma, 64, 0));
            ANV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&bg, k_gather_mfma, 64, 0));
        }
        // one block per work item in flight (two wavefronts for FP64, one for FP32)
        const int work = pl.nwave[3];
        pl.b_grid[0] = std::max(1, std::min(work, std::max(1, bs) * ncu));
        pl.b_grid[1] = std::max(1, std::min(work, std::max(1, bg) * ncu));
    }
    // right-hand sides per grid-step block: as many as the device's LDS per block
    // allows (160 KB on gfx950: all 16 FP64 right-hand sides of a 24^3 box in one
    // block, which reads whole 128-byte rows of the fold target; with the 64 KB
    // of older parts the FP64 grid step took 0.228 instead of 0.169 ms at N = 1e5)
    int dev = 0, lds_block = 0;
    ANV_HIP(hipGetDevice(&dev));
    ANV_HIP(hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int64_t kGridStepLds = std::max<int64_t>(65536, lds_block);
    const int64_t ex = pl.emax[0], ey = pl.emax[1], ez = pl.emax[2];
    pl.b_rsplit = 1;
    const int64_t exp = (ex + 3) & ~3, eyp = (ey + 3) & ~3, ezp = (ez + 3) & ~3;
    const int64_t el = int64_t(elem);
    while (pl.b_rsplit < RB && ((2 * ey * ez * (RB / pl.b_rsplit) + ey * eyp + ez * ezp) * el > kGridStepLds ||
                                (ex * ez * (RB / pl.b_rsplit) + ex * exp) * el > kGridStepLds))
        pl.b_rsplit *= 2;
    pl.b_ready = true;
}

namespace {

// one pass of up to RB right-hand sides; T = float (mixed precision: FP32
// MFMA spread, split-bf16 MFMA gather) or double (FP64 throughout)
template <class T>
void batched_pass_t(Plan& pl, const ColPtrs& cols, int rn, hipStream_t st) {
    constexpr bool f64 = sizeof(T) == sizeof(double);
    const int64_t N = pl.N;
    const bool prof = pl.profiling;
    const T* wts = f64 ? reinterpret_cast<const T*>(pl.wts64.p) : reinterpret_cast<const T*>(pl.wts32.p);
    T* xt = buf_as<T>(pl.xtb);
    T* fsb = buf_as<T>(pl.fsb);
    T* slab = buf_as<T>(pl.slabb);
    T* tgt = buf_as<T>(pl.tgtb);
    T* g1 = buf_as<T>(pl.g1b);
    T* hb = buf_as<T>(pl.hb);
    if (prof) pl.record_stage_event(st);
    hipLaunchKernelGGL(k_transpose_in<T>, dim3(nblk(N, 64)), dim3(256), 0, st, cols, rn, N, xt, pl.b_queue.p);
    if (prof) pl.record_stage_event(st);
    if (pl.nwave[3]) {
        if constexpr (f64)
            hipLaunchKernelGGL(k_spread_mfma64, dim3(pl.b_grid[0]), dim3(128), 0, st, pl.wave_items.p + pl.wave_off[3],
                               pl.nwave[3], pl.b_queue.p, pl.segs.p, pl.lstart.p, pl.lstart_off.p, pl.wins_d.p,
                               pl.alone.p, pl.wts64.p, pl.perm.p, xt, N, slab, tgt);
        else
            hipLaunchKernelGGL(k_spread_mfma, dim3(pl.b_grid[0]), dim3(64), 0, st, pl.wave_items.p + pl.wave_off[3],
                               pl.nwave[3], pl.b_queue.p, pl.segs.p, pl.lstart.p, pl.lstart_off.p, pl.wins_d.p,
                               pl.alone.p, pl.wts32.p, pl.perm.p, xt, N, slab, tgt);
    }
    if (pl.nb_items2)
        hipLaunchKernelGGL((k_spread_lane_b<8, 8, T>), dim3(nblk(int64_t(pl.nb_items2) * RB, 64)), dim3(64), 0, st,
                           pl.b_items.p, pl.nb_items2, pl.segs.p, pl.zq.p, wts, pl.perm.p, xt, N, slab);
    if (pl.nb_items1)
        hipLaunchKernelGGL((k_spread_lane_b<8, 1, T>), dim3(nblk(int64_t(pl.nb_items1) * RB, 64)), dim3(64), 0, st,
                           pl.b_items.p + pl.nb_items2, pl.nb_items1, pl.segs.p, pl.zq.p, wts, pl.perm.p, xt, N, slab);
    if (prof) pl.record_stage_event(st);
    if (pl.nflist)
        hipLaunchKernelGGL(k_fold_cols_b<T>, dim3(unsigned(pl.nflist)), dim3(256), 0, st, pl.wins_d.p, pl.P,
                           pl.nflist, pl.flist.p, pl.fold.p, pl.sbase.p, slab, tgt);
    if (prof) pl.record_stage_event(st);
    const int RH = RB / pl.b_rsplit;
    auto pad4 = [](int64_t e) { return (e + 3) & ~int64_t(3); };
    const size_t lds_yz = size_t(2 * pl.emax[1] * pl.emax[2] * RH + pl.emax[1] * pad4(pl.emax[1]) +
                                 pl.emax[2] * pad4(pl.emax[2])) * sizeof(T);
    // one block per (slice, window, right-hand-side slice), groups padded to a multiple of 8
    auto xcd_blocks = [&](int64_t ne) { return unsigned((ne * pl.P + 7) / 8 * 8 * pl.b_rsplit); };
    hipLaunchKernelGGL((k_fold_conv_yz_b<8, T>), dim3(xcd_blocks(pl.emax[0])), dim3(fold_conv_threads<T>()), lds_yz, st,
                       pl.wins_d.p,
                       pl.tmat.p, pl.crange.p, tgt, g1, RH, int(pl.emax[0]), int(pl.P));
    const size_t lds_x = size_t(pl.emax[0] * pl.emax[2] * RH + pl.emax[0] * pad4(pl.emax[0])) * sizeof(T);
    hipLaunchKernelGGL(k_conv_x_b<T>, dim3(xcd_blocks(pl.emax[1])), dim3(1024), lds_x, st, pl.wins_d.p, pl.tmat.p,
                       g1, hb, RH, int(pl.emax[1]), int(pl.P));
    if (prof) pl.record_stage_event(st);
    if (pl.nwave[3]) {
        if constexpr (f64)
            hipLaunchKernelGGL(k_gather_mfma64, dim3(pl.b_grid[1]), dim3(128), 0, st, pl.wave_items.p + pl.wave_off[3],
                               pl.nwave[3], pl.b_queue.p + 1, pl.segs.p, pl.lstart.p, pl.lstart_off.p,
                               pl.wins_d.p, pl.wts64.p, hb, N, fsb);
        else
            hipLaunchKernelGGL(k_gather_mfma, dim3(pl.b_grid[1]), dim3(64), 0, st, pl.wave_items.p + pl.wave_off[3],
                               pl.nwave[3], pl.b_queue.p + 1, pl.segs.p, pl.lstart.p, pl.lstart_off.p, pl.wins_d.p,
                               pl.wts32.p, hb, N, fsb);
    }
    if (pl.nb_items2)
        hipLaunchKernelGGL((k_gather_lane_b<8, 8, T>), dim3(nblk(int64_t(pl.nb_items2) * RB, 64)), dim3(64), 0, st,
                           pl.b_items.p, pl.nb_items2, pl.segs.p, pl.wins_d.p, pl.zq.p, wts, hb, N, fsb);
    if (pl.nb_items1)
        hipLaunchKernelGGL((k_gather_lane_b<8, 1, T>), dim3(nblk(int64_t(pl.nb_items1) * RB, 64)), dim3(64), 0, st,
                           pl.b_items.p + pl.nb_items2, pl.nb_items1, pl.segs.p, pl.wins_d.p, pl.zq.p, wts, hb, N, fsb);
    if (prof) pl.record_stage_event(st);
    hipLaunchKernelGGL(k_window_sum_b<T>, dim3(nblk(N, 64)), dim3(256), 0, st, fsb, pl.pos.p, pl.wins_d.p, pl.P, N,
                       rn, cols);
    if (prof) pl.record_stage_event(st);
    ANV_HIP(hipGetLastError());
}

void batched_pass(Plan& pl, const ColPtrs& cols, int rn, hipStream_t st) {
    if (pl.precision == ANOVA_PREC_FP64)
        batched_pass_t<double>(pl, cols, rn, st);
    else
        batched_pass_t<float>(pl, cols, rn, st);
}

}  // namespace

void enqueue_matvec_batched(Plan& pl, const double* x, int R, int64_t ldx, double* y, int64_t ldy, hipStream_t st) {
    ensure_batched_buffers(pl);
    for (int r0 = 0; r0 < R; r0 += RB) {
        const int rn = std::min(RB, R - r0);
        ColPtrs cols{};
        for (int r = 0; r < rn; ++r) {
            cols.x[r] = x + int64_t(r0 + r) * ldx;
            cols.y[r] = y + int64_t(r0 + r) * ldy;
        }
        batched_pass(pl, cols, rn, st);
    }
}

void enqueue_matvec_batched_cols(Plan& pl, const double* const* x, double* const* y, int R, hipStream_t st) {
    ensure_batched_buffers(pl);
    for (int r0 = 0; r0 < R; r0 += RB) {
        const int rn = std::min(RB, R - r0);
        ColPtrs cols{};
        for (int r = 0; r < rn; ++r) {
            cols.x[r] = x[r0 + r];
            cols.y[r] = y[r0 + r];
        }
        batched_pass(pl, cols, rn, st);
    }
}

// Shared launches batch the vectors of mixed-precision plans only: FP64 plans
// keep the one-vector kernels there, so that a served or grid solve on an FP64
// plan rounds exactly as the direct solve does.
static bool grouped_batching(const Plan& pl) { return pl.precision == ANOVA_PREC_MIXED && pl.W == 8; }

void enqueue_matvec_grouped(Plan* const* plans, const double* const* x, double* const* y, int n, hipStream_t st) {
    // same-plan vectors of batched plans: one batched pass per 16 of them;
    // the rest: shared one-vector launches
    std::vector<int> taken(n, 0);
    std::vector<Plan*> rp;
    std::vector<const double*> rx;
    std::vector<double*> ry;
    for (int i = 0; i < n; ++i) {
        if (taken[i]) continue;
        if (!grouped_batching(*plans[i])) {
            rp.push_back(plans[i]);
            rx.push_back(x[i]);
            ry.push_back(y[i]);
            taken[i] = 1;
            continue;
        }
        std::vector<const double*> gx;
        std::vector<double*> gy;
        for (int k = i; k < n; ++k)
            if (!taken[k] && plans[k] == plans[i]) {
                gx.push_back(x[k]);
                gy.push_back(y[k]);
                taken[k] = 1;
            }
        enqueue_matvec_batched_cols(*plans[i], gx.data(), gy.data(), int(gx.size()), st);
    }
    if (!rp.empty()) enqueue_matvec_multi(rp.data(), rx.data(), ry.data(), int(rp.size()), st);
}

}  // namespace anv
