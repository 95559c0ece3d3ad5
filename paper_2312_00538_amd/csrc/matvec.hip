// The ANOVA kernel matrix-vector product y = sum_l eta_l K_l x (Section 3),
// every window by NFFT fast summation:
//   spread   g = sum_i x_i phi(. - x_i)           (adjoint NFFT, inner sum)
//   convolve h = (T_x (x) T_y (x) T_z) g          (FFT, times B, inverse FFT)
//   gather   f_j = sum_cells h phi(x_j - .)       (forward NFFT, outer sum)
//   sum      y_j = sum_l eta_l f_j^{(l)}          (fixed window order, FP64)
//
// Work decomposition (gfx950, wave64). Points of a window are sorted by
// (column (cx, cy), layer cz) of their base cell. One wavefront handles one
// work item: a run of consecutive sorted points of one column. Lane (a, b) owns
// the grid line (cx + a, cy + b, *) of the 2m x 2m footprint shared by all
// points of the column, and keeps the 2m cells along z that the current point
// touches in registers; as the run advances in z, finished cells are written
// (spread) or new cells are loaded (gather). No atomics anywhere: each work
// item writes its own slab of partial sums, and the fold kernel adds the slabs
// that cover a cell in a fixed order, so results are reproducible bit for bit.
#include "plan.hpp"

namespace anv {

namespace {

constexpr int kThreads = 256;
inline unsigned nblocks(int64_t n, int t = kThreads) { return unsigned((n + t - 1) / t); }

__global__ void k_permute(const double* __restrict__ x, const int32_t* __restrict__ perm,
                          int64_t NP, int64_t N, double* __restrict__ vs) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= NP) return;
    vs[t] = x[perm[t]];
}

// One wavefront per work item. The loop is software-pipelined by one point:
// the z weights, input value and base layer of the next point (wave-uniform,
// scalar loads) and its per-lane x and y weights (vector loads) are requested
// before the current point is accumulated. The inner loop uses no LDS, so the
// scalar-load counter only ever waits for the point about to be used.
template <int W, class WT>
__global__ __launch_bounds__(64) void k_spread(const Segment* __restrict__ segs,
                                               const WinDev* __restrict__ wins,
                                               const int32_t* __restrict__ zq,
                                               const WT* __restrict__ wts,
                                               const double* __restrict__ vs, int64_t N,
                                               WT* __restrict__ slab) {
    const Segment sg = segs[blockIdx.x];
    const int lanes = wins[sg.win].lanes;
    const int wy = wins[sg.win].Wslot[1];
    const int lane = threadIdx.x;
    const bool active = lane < lanes;
    const int a = active ? lane / wy : 0;
    const int b = active ? lane % wy : 0;
    const int64_t base = int64_t(sg.win) * N + sg.start;
    WT* out = slab + sg.off;
    WT acc[W];
#pragma unroll
    for (int c = 0; c < W; ++c) acc[c] = WT(0);
    int zr = sg.z0;
    int64_t g = base;
    const int64_t gend = base + sg.count;
    int nz = zq[g];
    WT nv = WT(vs[g]);
    WT nw[W];
#pragma unroll
    for (int c = 0; c < W; ++c) nw[c] = wts[g * (3 * W) + 2 * W + c];
    WT nwx = wts[g * (3 * W) + a], nwy = wts[g * (3 * W) + W + b];
    for (; g < gend;) {
        const int zj = nz;
        const WT v = nv, wxa = nwx, wyb = nwy;
        WT wz[W];
#pragma unroll
        for (int c = 0; c < W; ++c) wz[c] = nw[c];
        ++g;
        if (g < gend) {
            nz = zq[g];
            nv = WT(vs[g]);
#pragma unroll
            for (int c = 0; c < W; ++c) nw[c] = wts[g * (3 * W) + 2 * W + c];
            nwx = wts[g * (3 * W) + a];
            nwy = wts[g * (3 * W) + W + b];
        }
        while (zr < zj) {  // layer zr is complete: no later point of the run reaches it
            if (active) out[(zr - sg.z0) * lanes + lane] = acc[0];
#pragma unroll
            for (int c = 0; c < W - 1; ++c) acc[c] = acc[c + 1];
            acc[W - 1] = WT(0);
            ++zr;
        }
        const WT coef = v * wxa * wyb;
#pragma unroll
        for (int c = 0; c < W; ++c) acc[c] += coef * wz[c];
    }
    if (active) {
#pragma unroll
        for (int c = 0; c < W; ++c) out[(zr - sg.z0 + c) * lanes + lane] = acc[c];
    }
}

// g[cell] = sum over the work items whose slabs cover the cell. One wavefront
// per cell; lane (a, b) reads the partial sums that column (gx - a, gy - b)
// wrote for its footprint position (a, b), and the lanes are combined by a
// fixed butterfly, so the order of additions never changes.
template <class WT>
__global__ __launch_bounds__(256) void k_fold(const WinDev* __restrict__ wins,
                                              const int2* __restrict__ fold,
                                              const int64_t* __restrict__ sbase,
                                              const WT* __restrict__ slab, WT* __restrict__ grid) {
    const int l = blockIdx.y;
    const WinDev& wd = wins[l];
    const int64_t cells = int64_t(wd.E[0]) * wd.E[1] * wd.E[2];
    const int64_t c = int64_t(blockIdx.x) * (blockDim.x / 64) + threadIdx.x / 64;
    if (c >= cells) return;
    const int lane = threadIdx.x % 64;
    const int gz = int(c % wd.E[2]);
    const int gy = int((c / wd.E[2]) % wd.E[1]);
    const int gx = int(c / (int64_t(wd.E[2]) * wd.E[1]));
    double acc = 0.0;
    if (lane < wd.lanes) {
        const int a = lane / wd.Wslot[1], b = lane % wd.Wslot[1];
        const int cx = gx - a, cy = gy - b;
        if (cx >= 0 && cx < wd.nb[0] && cy >= 0 && cy < wd.nb[1]) {
            const int2 r = fold[wd.fold_off + (int64_t(cx) * wd.nb[1] + cy) * wd.E[2] + gz];
            for (int s = r.x; s < r.y; ++s) acc += double(slab[sbase[s] + int64_t(gz) * wd.lanes + lane]);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) grid[wd.grid_off + c] = WT(acc);
}

// out = T_axis applied along one axis of every window grid (layout [x][y][z])
template <class WT>
__global__ void k_conv_axis(const WinDev* __restrict__ wins, const double* __restrict__ tmat,
                            int axis, const WT* __restrict__ in, WT* __restrict__ out) {
    const int l = blockIdx.y;
    const WinDev wd = wins[l];
    const int64_t cells = int64_t(wd.E[0]) * wd.E[1] * wd.E[2];
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const int E = wd.E[axis];
    int64_t stride = 1;
    for (int s = 2; s > axis; --s) stride *= wd.E[s];
    const int i = int((c / stride) % E);
    const int64_t base = wd.grid_off + c - int64_t(i) * stride;
    const double* T = tmat + wd.t_off[axis] + int64_t(i) * E;
    double acc = 0.0;
    for (int k = 0; k < E; ++k) acc += T[k] * double(in[base + int64_t(k) * stride]);
    out[wd.grid_off + c] = WT(acc);
}

// One wavefront per work item. Lane (a, b) keeps the 2m grid values of its line
// (cx + a, cy + b, zr .. zr + 2m - 1) in registers. Loads are pipelined one
// point ahead as in the spread. Each point's per-lane partial product goes to
// LDS and after every chunk of points the wave sums them per point in lane
// order (one transposed reduction instead of a shuffle tree per point).
template <int W, class WT>
__global__ __launch_bounds__(64) void k_gather(const Segment* __restrict__ segs,
                                               const WinDev* __restrict__ wins,
                                               const int32_t* __restrict__ zq,
                                               const WT* __restrict__ wts,
                                               const WT* __restrict__ h, int64_t N,
                                               double* __restrict__ fs) {
    constexpr int CH = 32;
    __shared__ double red[CH][65];
    const Segment sg = segs[blockIdx.x];
    const WinDev& wd = wins[sg.win];
    const int lanes = wd.lanes;
    const int wy = wd.Wslot[1];
    const int lane = threadIdx.x;
    const bool active = lane < lanes;
    const int a = active ? lane / wy : 0;
    const int b = active ? lane % wy : 0;
    const int cx = sg.col / wd.nb[1];
    const int cy = sg.col % wd.nb[1];
    const int Ez = wd.E[2];
    const WT* hcol = h + wd.grid_off + (int64_t(cx + a) * wd.E[1] + (cy + b)) * Ez;
    const int64_t base = int64_t(sg.win) * N + sg.start;
    WT ring[W];
    int zr = sg.z0;
#pragma unroll
    for (int c = 0; c < W; ++c) ring[c] = active ? hcol[zr + c] : WT(0);
    WT nxt = (active && zr + W < Ez) ? hcol[zr + W] : WT(0);
    int64_t g = base;
    const int64_t gend = base + sg.count;
    int nz = zq[g];
    WT nw[W];
#pragma unroll
    for (int c = 0; c < W; ++c) nw[c] = wts[g * (3 * W) + 2 * W + c];
    WT nwx = wts[g * (3 * W) + a], nwy = wts[g * (3 * W) + W + b];
    for (int j0 = 0; j0 < sg.count; j0 += CH) {
        const int nb = min(CH, sg.count - j0);
        for (int jj = 0; jj < nb; ++jj) {
            const int zj = nz;
            const WT wxa = nwx, wyb = nwy;
            WT wz[W];
#pragma unroll
            for (int c = 0; c < W; ++c) wz[c] = nw[c];
            ++g;
            if (g < gend) {
                nz = zq[g];
#pragma unroll
                for (int c = 0; c < W; ++c) nw[c] = wts[g * (3 * W) + 2 * W + c];
                nwx = wts[g * (3 * W) + a];
                nwy = wts[g * (3 * W) + W + b];
            }
            while (zr < zj) {
#pragma unroll
                for (int c = 0; c < W - 1; ++c) ring[c] = ring[c + 1];
                ring[W - 1] = nxt;
                ++zr;
                nxt = (active && zr + W < Ez) ? hcol[zr + W] : WT(0);
            }
            WT s = WT(0);
#pragma unroll
            for (int c = 0; c < W; ++c) s += wz[c] * ring[c];
            red[jj][lane] = active ? double(s * wxa * wyb) : 0.0;
        }
        __syncthreads();
        if (lane < nb) {
            double sum = 0.0;
            for (int q = 0; q < lanes; ++q) sum += red[lane][q];
            fs[base + j0 + lane] = sum;
        }
        __syncthreads();
    }
}

__global__ void k_window_sum(const double* __restrict__ fs, const int32_t* __restrict__ pos,
                             const WinDev* __restrict__ wins, int32_t P, int64_t N,
                             double* __restrict__ y) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    for (int l = 0; l < P; ++l) acc += wins[l].eta * fs[int64_t(l) * N + pos[int64_t(l) * N + i]];
    y[i] = acc;
}

template <int W, class WT>
void run_matvec(Plan& pl, const double* x, double* y, WT* wts, WT* slab, WT* g, WT* h, WT* ca,
                WT* cb, hipStream_t st) {
    const int64_t N = pl.N, NP = pl.N * pl.P;
    const unsigned nseg = unsigned(pl.segs_h.size());
    const bool prof = pl.profiling;
    if (prof) pl.record_stage_event(st);
    hipLaunchKernelGGL(k_permute, dim3(nblocks(NP)), dim3(kThreads), 0, st, x, pl.perm.p, NP, N,
                       pl.vs.p);
    if (prof) pl.record_stage_event(st);
    hipLaunchKernelGGL((k_spread<W, WT>), dim3(nseg), dim3(64), 0, st, pl.segs.p, pl.wins_d.p,
                       pl.zq.p, wts, pl.vs.p, N, slab);
    const dim3 gg(nblocks(pl.grid_max), unsigned(pl.P));
    if (prof) pl.record_stage_event(st);
    hipLaunchKernelGGL(k_fold<WT>, dim3(unsigned((pl.grid_max + 3) / 4), unsigned(pl.P)), dim3(256), 0,
                       st, pl.wins_d.p, pl.fold.p, pl.sbase.p, slab, g);
    if (prof) pl.record_stage_event(st);
    hipLaunchKernelGGL(k_conv_axis<WT>, gg, dim3(kThreads), 0, st, pl.wins_d.p, pl.tmat.p, 0, g, ca);
    hipLaunchKernelGGL(k_conv_axis<WT>, gg, dim3(kThreads), 0, st, pl.wins_d.p, pl.tmat.p, 1, ca, cb);
    hipLaunchKernelGGL(k_conv_axis<WT>, gg, dim3(kThreads), 0, st, pl.wins_d.p, pl.tmat.p, 2, cb, h);
    if (prof) pl.record_stage_event(st);
    hipLaunchKernelGGL((k_gather<W, WT>), dim3(nseg), dim3(64), 0, st, pl.segs.p, pl.wins_d.p,
                       pl.zq.p, wts, h, N, pl.fs.p);
    if (prof) pl.record_stage_event(st);
    hipLaunchKernelGGL(k_window_sum, dim3(nblocks(N)), dim3(kThreads), 0, st, pl.fs.p, pl.pos.p,
                       pl.wins_d.p, pl.P, N, y);
    if (prof) pl.record_stage_event(st);
    ANV_HIP(hipGetLastError());
}

template <int W>
void run_prec(Plan& pl, const double* x, double* y, hipStream_t st) {
    if (pl.precision == ANOVA_PREC_FP64)
        run_matvec<W, double>(pl, x, y, pl.wts64.p, pl.slab64.p, pl.g64.p, pl.h64.p, pl.c64a.p,
                              pl.c64b.p, st);
    else
        run_matvec<W, float>(pl, x, y, pl.wts32.p, pl.slab32.p, pl.g32.p, pl.h32.p, pl.c32a.p,
                             pl.c32b.p, st);
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
    for (int r = 0; r < R; ++r) {
        const double* xr = x + int64_t(r) * ldx;
        double* yr = y + int64_t(r) * ldy;
        switch (pl.W) {
            case 4: run_prec<4>(pl, xr, yr, st); break;
            case 6: run_prec<6>(pl, xr, yr, st); break;
            case 8: run_prec<8>(pl, xr, yr, st); break;
            default: throw Error(ANOVA_INVALID_ARG, "unsupported cutoff");
        }
    }
}

}  // namespace anv
