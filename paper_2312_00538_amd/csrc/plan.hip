// Plan construction (setup of the fast summation, Section 3): per window, map
// its features onto the torus box, bin the points into base cells of the
// oversampled grid, sort them by (column, layer), evaluate their Kaiser-Bessel
// weights once, and lay out the wavefront work items of the spreading and
// gathering kernels.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "plan.hpp"

namespace anv {

namespace {

constexpr int kThreads = 256;

// xw[(i*P + l)*3 + s] = X[i, feature of slot s of window l] (0 for a dummy slot)
__global__ void k_window_coords(const double* __restrict__ X, int64_t N, int64_t ldx,
                                const int32_t* __restrict__ sfeat, int32_t P,
                                double* __restrict__ xw) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t total = N * P * 3;
    if (t >= total) return;
    int64_t i = t / (3 * P);
    int ls = int(t % (3 * P));
    int f = sfeat[ls];
    xw[t] = f >= 0 ? X[i * ldx + f] : 0.0;
}

// partial min/max of one (window, slot) column over a chunk of points
__global__ void k_minmax(const double* __restrict__ xw, int64_t N, int32_t P, int64_t chunk,
                         double* __restrict__ part) {
    __shared__ double smin[kThreads], smax[kThreads];
    int ls = blockIdx.y;
    int64_t i0 = blockIdx.x * chunk;
    int64_t i1 = min(N, i0 + chunk);
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        double v = xw[i * 3 * P + ls];
        lo = fmin(lo, v);
        hi = fmax(hi, v);
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[(int64_t(ls) * gridDim.x + blockIdx.x) * 2 + 0] = smin[0];
        part[(int64_t(ls) * gridDim.x + blockIdx.x) * 2 + 1] = smax[0];
    }
}

struct AxisMap {
    double center, scale;
    int32_t real;
    int32_t pad;
};

// torus coordinate u = (x - center) * scale; grid position nu = n_os * u;
// base cell q = floor(nu) - m + 1 (first of the 2m cells within the support);
// fractional part t = nu - floor(nu) in [0, 1).
__global__ void k_bin(const double* __restrict__ xw, int64_t N, int32_t P,
                      const AxisMap* __restrict__ amap, int32_t n_os, int32_t m,
                      int32_t* __restrict__ q, double* __restrict__ tf) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * P) return;
    int l = int(t / N);
    int64_t i = t % N;
    for (int s = 0; s < 3; ++s) {
        AxisMap am = amap[l * 3 + s];
        int qq = 0;
        double fr = 0.0;
        if (am.real) {
            double u = (xw[(i * P + l) * 3 + s] - am.center) * am.scale;
            double nu = double(n_os) * u;
            double fl = floor(nu);
            qq = int(fl) - m + 1;
            fr = nu - fl;
        }
        q[t * 3 + s] = qq;
        tf[t * 3 + s] = fr;
    }
}

// per (window, slot): min and max base cell, reduced per block before one atomic
__global__ void k_qext(const int32_t* __restrict__ q, int64_t N, int32_t* __restrict__ qext) {
    __shared__ int smin[256], smax[256];
    const int ls = blockIdx.y;  // window * 3 + slot
    const int l = ls / 3, s = ls % 3;
    int lo = INT32_MAX, hi = INT32_MIN;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x) {
        int v = q[(int64_t(l) * N + i) * 3 + s];
        lo = min(lo, v);
        hi = max(hi, v);
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            smin[threadIdx.x] = min(smin[threadIdx.x], smin[threadIdx.x + k]);
            smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + k]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMin(&qext[ls * 2 + 0], smin[0]);
        atomicMax(&qext[ls * 2 + 1], smax[0]);
    }
}

__global__ void k_keys(const int32_t* __restrict__ q, int64_t N, int32_t P,
                       const int32_t* __restrict__ qmin, const int32_t* __restrict__ nbv,
                       uint32_t* __restrict__ keys, int32_t* __restrict__ vals) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * P) return;
    int l = int(t / N);
    int64_t i = t % N;
    uint32_t cx = uint32_t(q[t * 3 + 0] - qmin[l * 3 + 0]);
    uint32_t cy = uint32_t(q[t * 3 + 1] - qmin[l * 3 + 1]);
    uint32_t cz = uint32_t(q[t * 3 + 2] - qmin[l * 3 + 2]);
    keys[t] = (cx * uint32_t(nbv[l * 3 + 1]) + cy) * uint32_t(nbv[l * 3 + 2]) + cz;
    vals[t] = int32_t(i);
}

// normalised Kaiser-Bessel window phi(u)/phi(0), |u| <= m (grid cells)
__device__ double kb_dev(double u, int m, double b) {
    double s2 = double(m) * m - u * u;
    double s = s2 > 0.0 ? sqrt(s2) : 0.0;
    double v = s > 0.0 ? sinh(b * s) / s : b;
    return v / (sinh(b * m) / m);
}

template <class WT>
__global__ void k_weights(const int32_t* __restrict__ perm, const int32_t* __restrict__ q,
                          const double* __restrict__ tf, int64_t N, int32_t P,
                          const int32_t* __restrict__ qmin, const int32_t* __restrict__ wslot,
                          int32_t W, int32_t m, double b, int32_t* __restrict__ pos,
                          int32_t* __restrict__ zq, WT* __restrict__ wts) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * P) return;
    int l = int(t / N);
    int64_t i = perm[t];
    int64_t src = int64_t(l) * N + i;
    pos[src] = int32_t(t - int64_t(l) * N);
    zq[t] = q[src * 3 + 2] - qmin[l * 3 + 2];
    const int RECG = rec_stride(W, int(sizeof(WT)));
    for (int e = 3 * W; e < RECG; ++e) wts[t * RECG + e] = WT(0);
    for (int s = 0; s < 3; ++s) {
        WT* w = wts + t * RECG + s * W;
        if (wslot[l * 3 + s] == 1) {
            w[0] = WT(1);
            for (int a = 1; a < W; ++a) w[a] = WT(0);
        } else {
            double fr = tf[src * 3 + s];
            for (int a = 0; a < W; ++a) w[a] = WT(kb_dev(fr + double(m - 1 - a), m, b));
        }
    }
}

template <class T>
void upload(DevBuf<T>& buf, const std::vector<T>& h, hipStream_t st) {
    buf.alloc(h.size());
    ANV_HIP(hipMemcpyAsync(buf.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

inline unsigned nblocks(int64_t n, int t = kThreads) { return unsigned((n + t - 1) / t); }

}  // namespace

int64_t Plan::device_bytes() const {
    return int64_t(wins_d.bytes() + sbase.bytes() + wave_items.bytes() + lstart.bytes() + lstart_off.bytes() +
                   alone.bytes() + flist.bytes() + crange.bytes() + perm.bytes() + pos.bytes() + zq.bytes() + wts64.bytes() +
                   wts32.bytes() + segs.bytes() + fold.bytes() + tmat.bytes() + xw.bytes() +
                   vs.bytes() + fs.bytes() + g64.bytes() + h64.bytes() + c64a.bytes() +
                   c64b.bytes() + g32.bytes() + h32.bytes() + c32a.bytes() + c32b.bytes() +
                   slab64.bytes() + slab32.bytes() + xtb.bytes() + fsb.bytes() + slabb.bytes() +
                   tgtb.bytes() + g1b.bytes() + hb.bytes() + b_items.bytes() + b_queue.bytes());
}

Plan* create_plan(const double* X, int64_t N, int32_t d, int64_t ldx, const int32_t* windows,
                  int32_t P, const double* sigma, const double* eta, const anova_opts* opts,
                  hipStream_t st) {
    ANV_CHECK(X != nullptr && windows != nullptr && sigma != nullptr, "NULL argument");
    ANV_CHECK(N >= 1 && d >= 1 && P >= 1, "need N >= 1, d >= 1, P >= 1");
    ANV_CHECK(ldx >= d, "ldx < d");
    ANV_CHECK(N * int64_t(P) < (int64_t(1) << 31), "N * P too large");
    anova_opts o;
    anova_opts_default(&o);
    if (opts) {
        ANV_CHECK(opts->version == ANOVA_OPTS_VERSION, "anova_opts.version mismatch");
        o = *opts;
    }
    ANV_CHECK(o.n_bw >= 4 && o.n_bw % 2 == 0 && o.n_bw <= 256, "n_bw must be even, 4..256");
    ANV_CHECK(o.oversample >= 2 && o.oversample <= 4, "oversample must be 2..4");
    ANV_CHECK(o.cutoff_m >= 2 && o.cutoff_m <= 4, "cutoff_m must be 2..4");
    ANV_CHECK(o.eps_b > 0.0 && o.eps_b < 0.5, "eps_b must be in (0, 1/2)");
    ANV_CHECK(o.reg_p <= 30, "reg_p must be <= 30");
    ANV_CHECK(o.precision == ANOVA_PREC_FP64 || o.precision == ANOVA_PREC_MIXED, "bad precision");

    auto pl = std::make_unique<Plan>();
    pl->N = N;
    pl->d = d;
    pl->P = P;
    pl->prm.n_bw = o.n_bw;
    pl->prm.n_os = o.n_bw * o.oversample;
    pl->prm.m = o.cutoff_m;
    pl->prm.eps_b = o.eps_b;
    pl->prm.reg_p = o.reg_p;
    pl->W = 2 * o.cutoff_m;
    pl->precision = o.precision;
    pl->seg_points = o.seg_points > 0 ? o.seg_points : 768;
    pl->batch_min_rhs = o.batch_min_rhs == 0 ? 2 : o.batch_min_rhs;
    const int W = pl->W, m = pl->prm.m, n_os = pl->prm.n_os;
    pl->win.assign(windows, windows + 3 * P);
    pl->sigma.assign(sigma, sigma + P);
    pl->eta.assign(P, 1.0);
    if (eta) pl->eta.assign(eta, eta + P);
    pl->slot_feat.resize(P);
    for (int l = 0; l < P; ++l) {
        std::vector<int> f;
        for (int a = 0; a < 3; ++a) {
            int v = windows[3 * l + a];
            if (v < 0) continue;
            ANV_CHECK(v < d, "window feature index out of range");
            for (int u : f) ANV_CHECK(u != v, "repeated feature in a window");
            f.push_back(v);
        }
        ANV_CHECK(!f.empty(), "empty window");
        ANV_CHECK(std::isfinite(pl->sigma[l]) && pl->sigma[l] > 0.0, "sigma must be > 0");
        ANV_CHECK(std::isfinite(pl->eta[l]), "eta must be finite");
        // the last feature takes the z slot (the register-resident axis of the kernels)
        std::array<int32_t, 3> sf = {-1, -1, -1};
        int off = 3 - int(f.size());
        for (size_t a = 0; a < f.size(); ++a) sf[off + a] = f[a];
        pl->slot_feat[l] = sf;
    }

    // 1. windowed coordinates and their ranges
    std::vector<int32_t> sfeat(3 * P);
    for (int l = 0; l < P; ++l)
        for (int s = 0; s < 3; ++s) sfeat[3 * l + s] = pl->slot_feat[l][s];
    DevBuf<int32_t> sfeat_d;
    upload(sfeat_d, sfeat, st);
    pl->xw.alloc(size_t(N) * P * 3);
    hipLaunchKernelGGL(k_window_coords, dim3(nblocks(N * P * 3)), dim3(kThreads), 0, st, X, N, ldx,
                       sfeat_d.p, P, pl->xw.p);
    ANV_HIP(hipGetLastError());
    const int64_t chunk = 1 << 15;
    const int nchunk = int((N + chunk - 1) / chunk);
    DevBuf<double> part;
    part.alloc(size_t(nchunk) * 3 * P * 2);
    hipLaunchKernelGGL(k_minmax, dim3(nchunk, 3 * P), dim3(kThreads), 0, st, pl->xw.p, N, P, chunk,
                       part.p);
    ANV_HIP(hipGetLastError());
    std::vector<double> parth(part.n);
    ANV_HIP(hipMemcpyAsync(parth.data(), part.p, part.bytes(), hipMemcpyDeviceToHost, st));
    ANV_HIP(hipStreamSynchronize(st));

    // 2. per-axis coefficients (host, FP64)
    pl->axes.resize(P);
    std::vector<AxisMap> amap(3 * P);
    for (int l = 0; l < P; ++l) {
        for (int s = 0; s < 3; ++s) {
            AxisMap am{0.0, 1.0, 0, 0};
            if (pl->slot_feat[l][s] >= 0) {
                double lo = INFINITY, hi = -INFINITY;
                for (int c = 0; c < nchunk; ++c) {
                    lo = std::min(lo, parth[((3 * l + s) * size_t(nchunk) + c) * 2 + 0]);
                    hi = std::max(hi, parth[((3 * l + s) * size_t(nchunk) + c) * 2 + 1]);
                }
                ANV_CHECK(std::isfinite(lo) && std::isfinite(hi), "X contains NaN or Inf");
                pl->axes[l][s] = build_axis(lo, hi, pl->sigma[l], pl->prm);
                pl->max_kerr = std::max(pl->max_kerr, pl->axes[l][s].kerr);
                am = AxisMap{pl->axes[l][s].center, pl->axes[l][s].scale, 1, 0};
            }
            amap[3 * l + s] = am;
        }
    }

    // 3. binning
    DevBuf<AxisMap> amap_d;
    upload(amap_d, amap, st);
    DevBuf<int32_t> qbuf, qext;
    DevBuf<double> tbuf;
    qbuf.alloc(size_t(N) * P * 3);
    tbuf.alloc(size_t(N) * P * 3);
    std::vector<int32_t> qext_h(6 * P);
    for (int i = 0; i < 3 * P; ++i) {
        qext_h[2 * i] = INT32_MAX;
        qext_h[2 * i + 1] = INT32_MIN;
    }
    upload(qext, qext_h, st);
    hipLaunchKernelGGL(k_bin, dim3(nblocks(N * P)), dim3(kThreads), 0, st, pl->xw.p, N, P, amap_d.p,
                       n_os, m, qbuf.p, tbuf.p);
    ANV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_qext, dim3(unsigned(std::min<int64_t>(64, (N + 255) / 256)), unsigned(3 * P)),
                       dim3(256), 0, st, qbuf.p, N, qext.p);
    ANV_HIP(hipGetLastError());
    ANV_HIP(hipMemcpyAsync(qext_h.data(), qext.p, qext.bytes(), hipMemcpyDeviceToHost, st));
    ANV_HIP(hipStreamSynchronize(st));

    std::vector<int32_t> qmin(3 * P), nbv(3 * P), wsl(3 * P);
    pl->wins_h.resize(P);
    int64_t goff = 0, toff = 0;
    std::vector<double> tm_h;
    for (int l = 0; l < P; ++l) {
        WinDev& wd = pl->wins_h[l];
        std::memset(&wd, 0, sizeof(wd));
        for (int s = 0; s < 3; ++s) {
            bool real = pl->slot_feat[l][s] >= 0;
            int lo = qext_h[(3 * l + s) * 2], hi = qext_h[(3 * l + s) * 2 + 1];
            if (!real) lo = hi = 0;
            int ws = real ? W : 1;
            wd.Wslot[s] = ws;
            wd.nb[s] = hi - lo + 1;
            wd.E[s] = hi - lo + ws;
            ANV_CHECK(wd.E[s] <= n_os, "occupied grid extent exceeds the FFT length");
            qmin[3 * l + s] = lo;
            nbv[3 * l + s] = wd.nb[s];
            wsl[3 * l + s] = ws;
            wd.t_off[s] = toff;
            const int E = wd.E[s];
            tm_h.resize(size_t(toff) + size_t(E) * E);
            for (int i = 0; i < E; ++i)
                for (int k = 0; k < E; ++k)
                    tm_h[toff + size_t(i) * E + k] = real ? pl->axes[l][s].circ[std::abs(i - k)] : 1.0;
            toff += int64_t(E) * E;
        }
        wd.lanes = wd.Wslot[0] * wd.Wslot[1];
        for (int s2 = 0; s2 < 3; ++s2) pl->emax[s2] = std::max(pl->emax[s2], wd.E[s2]);
        wd.grid_off = goff;
        int64_t cells = int64_t(wd.E[0]) * wd.E[1] * wd.E[2];
        goff += cells;
        pl->grid_max = std::max(pl->grid_max, cells);
        wd.eta = pl->eta[l];
        ANV_CHECK(int64_t(wd.nb[0]) * wd.nb[1] * wd.nb[2] < (int64_t(1) << 31), "too many cells");
    }
    pl->grid_total = goff;
    pl->tmat_total = toff;
    {
        const int64_t ey = pl->emax[1], ez = pl->emax[2], ex = pl->emax[0];
        const int64_t lds_yz = (2 * ey * ez + ey * ey + ez * ez) * 8, lds_x = (ex * ez + ex * ex) * 8;
        for (int l = 0; l < P; ++l) ANV_CHECK(pl->wins_h[l].nb[1] <= 64, "occupied grid box too large");
        ANV_CHECK(lds_yz <= 65536 && lds_x <= 65536,
                  "occupied grid box too large for the LDS-resident grid step (reduce n_bw or raise eps_b)");
    }
    upload(pl->tmat, tm_h, st);

    // 4. sort points of each window by (column, layer); stable, so ties keep point order
    DevBuf<int32_t> qmin_d, nbv_d, wsl_d;
    upload(qmin_d, qmin, st);
    upload(nbv_d, nbv, st);
    upload(wsl_d, wsl, st);
    DevBuf<uint32_t> keys, keys_sorted;
    DevBuf<int32_t> vals;
    keys.alloc(size_t(N) * P);
    keys_sorted.alloc(size_t(N) * P);
    vals.alloc(size_t(N) * P);
    pl->perm.alloc(size_t(N) * P);
    hipLaunchKernelGGL(k_keys, dim3(nblocks(N * P)), dim3(kThreads), 0, st, qbuf.p, N, P, qmin_d.p,
                       nbv_d.p, keys.p, vals.p);
    ANV_HIP(hipGetLastError());
    size_t temp_bytes = 0;
    ANV_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, keys.p, keys_sorted.p, vals.p,
                                               pl->perm.p, int(N), 0, 32, st));
    DevBuf<char> temp;
    temp.alloc(temp_bytes);
    for (int l = 0; l < P; ++l) {
        int64_t ncell = int64_t(nbv[3 * l]) * nbv[3 * l + 1] * nbv[3 * l + 2];
        int endbit = 1;
        while ((int64_t(1) << endbit) < ncell) ++endbit;
        size_t tb = temp_bytes;
        ANV_HIP(hipcub::DeviceRadixSort::SortPairs(temp.p, tb, keys.p + size_t(l) * N,
                                                   keys_sorted.p + size_t(l) * N, vals.p + size_t(l) * N,
                                                   pl->perm.p + size_t(l) * N, int(N), 0, endbit, st));
    }
    std::vector<uint32_t> ks(size_t(N) * P);
    ANV_HIP(hipMemcpyAsync(ks.data(), keys_sorted.p, keys_sorted.bytes(), hipMemcpyDeviceToHost, st));

    // 5. weights, inverse permutation, base layer per sorted point
    pl->pos.alloc(size_t(N) * P);
    pl->zq.alloc(size_t(N) * P);
    const double bkb = M_PI * (2.0 - double(pl->prm.n_bw) / n_os);
    if (pl->precision == ANOVA_PREC_FP64) {
        pl->wts64.alloc(size_t(N) * P * rec_stride(W, 8));
        hipLaunchKernelGGL(k_weights<double>, dim3(nblocks(N * P)), dim3(kThreads), 0, st, pl->perm.p,
                           qbuf.p, tbuf.p, N, P, qmin_d.p, wsl_d.p, W, m, bkb, pl->pos.p, pl->zq.p,
                           pl->wts64.p);
    } else {
        pl->wts32.alloc(size_t(N) * P * rec_stride(W, 4));
        hipLaunchKernelGGL(k_weights<float>, dim3(nblocks(N * P)), dim3(kThreads), 0, st, pl->perm.p,
                           qbuf.p, tbuf.p, N, P, qmin_d.p, wsl_d.p, W, m, bkb, pl->pos.p, pl->zq.p,
                           pl->wts32.p);
    }
    ANV_HIP(hipGetLastError());
    ANV_HIP(hipStreamSynchronize(st));

    // 6. work items: runs of at most seg_points sorted points of one column, and
    //    for every (column, layer) the contiguous range of items that touch it
    //    1- and 2-feature windows run one lane per item: their items are sized so
    //    that about 32K lanes (512 wavefronts) share the points, 8..128 points each
    {
        int64_t lane_points = 0;
        for (int l = 0; l < P; ++l) {
            int dw = 0;
            for (int s2 = 0; s2 < 3; ++s2) dw += pl->slot_feat[l][s2] >= 0;
            if (dw < 3) lane_points += N;
        }
        pl->seg_points_lane = int32_t(std::min<int64_t>(128, std::max<int64_t>(8, lane_points / 32768)));
    }
    std::vector<int2> fold_h;
    int64_t slab_off = 0, col_total = 0;
    for (int l = 0; l < P; ++l) {
        WinDev& wd = pl->wins_h[l];
        const int nbz = wd.nb[2], Ez = wd.E[2];
        const int64_t ncol = int64_t(wd.nb[0]) * wd.nb[1];
        wd.col_off = col_total;
        col_total += ncol;
        wd.fold_off = int64_t(fold_h.size());
        fold_h.resize(fold_h.size() + size_t(ncol) * Ez, int2{0, 0});
        const uint32_t* kk = ks.data() + size_t(l) * N;
        int dwl = 0;
        for (int s2 = 0; s2 < 3; ++s2) dwl += pl->slot_feat[l][s2] >= 0;
        const int sp = dwl == 3 ? pl->seg_points : pl->seg_points_lane;
        int64_t j = 0;
        while (j < N) {
            int64_t col = kk[j] / nbz;
            int64_t cb = int64_t(pl->segs_h.size());
            while (j < N && int64_t(kk[j] / nbz) == col) {
                Segment sg;
                sg.win = l;
                sg.col = int32_t(col);
                sg.start = int32_t(j);
                sg.z0 = int32_t(kk[j] % nbz);
                int32_t cnt = 0;
                // at most kItemLayers layers per item, so that a wavefront holds
                // the item's layer starts in one register (one entry per lane)
                while (j < N && int64_t(kk[j] / nbz) == col && cnt < sp &&
                       int32_t(kk[j] % nbz) - sg.z0 < kItemLayers) {
                    ++j;
                    ++cnt;
                }
                sg.count = cnt;
                sg.z1 = int32_t(kk[j - 1] % nbz);
                sg.off = slab_off;
                slab_off += int64_t(sg.z1 - sg.z0 + W) * wd.lanes;
                pl->segs_h.push_back(sg);
            }
            int64_t ce = int64_t(pl->segs_h.size());
            int64_t sb = cb, se = cb;
            for (int L = 0; L < Ez; ++L) {
                while (sb < ce && pl->segs_h[sb].z1 + W - 1 < L) ++sb;
                while (se < ce && pl->segs_h[se].z0 <= L) ++se;
                fold_h[wd.fold_off + col * Ez + L] = (sb < se) ? int2{int(sb), int(se)} : int2{0, 0};
            }
        }
    }
    ANV_CHECK(pl->segs_h.size() < (size_t(1) << 31), "too many work items");
    {
        // per window kind, work items sorted by length (longest first) so that the
        // items sharing a wavefront have similar lengths; packed 64/W or 64 per wave
        std::vector<int32_t> items;
        for (int kind = 3; kind >= 1; --kind) {
            std::vector<int32_t> ids;
            for (size_t i = 0; i < pl->segs_h.size(); ++i) {
                int l = pl->segs_h[i].win;
                int dw = 0;
                for (int s2 = 0; s2 < 3; ++s2) dw += pl->slot_feat[l][s2] >= 0;
                if (dw == kind) ids.push_back(int32_t(i));
            }
            std::stable_sort(ids.begin(), ids.end(), [&](int32_t u, int32_t v) {
                return pl->segs_h[u].count > pl->segs_h[v].count;
            });
            const int per = kind == 3 ? 1 : 64;
            pl->wave_off[kind] = int64_t(items.size());
            pl->nwave[kind] = int32_t((ids.size() + per - 1) / per);
            for (int32_t w = 0; w < pl->nwave[kind]; ++w)
                for (int q = 0; q < per; ++q) {
                    size_t idx = size_t(w) * per + q;
                    items.push_back(idx < ids.size() ? ids[idx] : -1);
                }
        }
        if (items.empty()) items.push_back(-1);
        upload(pl->wave_items, items, st);
        // layer starts of 3-feature items
        std::vector<int32_t> lso(pl->segs_h.size(), 0), lsv;
        for (size_t i = 0; i < pl->segs_h.size(); ++i) {
            const Segment& sgi = pl->segs_h[i];
            int l = sgi.win;
            int dw = 0;
            for (int s2 = 0; s2 < 3; ++s2) dw += pl->slot_feat[l][s2] >= 0;
            if (dw != 3) continue;
            lso[i] = int32_t(lsv.size());
            const uint32_t* kk = ks.data() + size_t(l) * N + sgi.start;
            const int nbz = pl->wins_h[l].nb[2];
            int j2 = 0;
            for (int z = sgi.z0; z <= sgi.z1 + 1; ++z) {
                while (j2 < sgi.count && int(kk[j2] % nbz) < z) ++j2;
                lsv.push_back(j2);
            }
        }
        if (lsv.empty()) lsv.push_back(0);
        upload(pl->lstart, lsv, st);
        upload(pl->lstart_off, lso, st);
        // items alone in their column; fold entries of the other columns; column layer ranges
        std::vector<uint8_t> al(pl->segs_h.size(), 0);
        std::vector<int2> cr(size_t(col_total + 1), int2{1, 0});
        // fold entries of 3-feature windows first, then those of 1- and 2-feature
        // windows (whose cells gather many short items and are folded by blocks)
        std::vector<int64_t> fl, fl_lane;
        size_t i0 = 0;
        while (i0 < pl->segs_h.size()) {
            size_t i1 = i0;
            while (i1 < pl->segs_h.size() && pl->segs_h[i1].win == pl->segs_h[i0].win &&
                   pl->segs_h[i1].col == pl->segs_h[i0].col)
                ++i1;
            const Segment& s0 = pl->segs_h[i0];
            const WinDev& wd = pl->wins_h[s0.win];
            int dw = 0;
            for (int s2 = 0; s2 < 3; ++s2) dw += pl->slot_feat[s0.win][s2] >= 0;
            const int64_t cidx = wd.col_off + s0.col;
            if (dw == 3 && i1 - i0 == 1) {
                al[i0] = 1;
                cr[cidx] = int2{s0.z0, s0.z1 + W - 1};
            } else {
                cr[cidx] = int2{0, wd.E[2] - 1};
                for (int L = 0; L < wd.E[2]; ++L)
                    (dw == 3 ? fl : fl_lane).push_back(wd.fold_off + int64_t(s0.col) * wd.E[2] + L);
            }
            i0 = i1;
        }
        upload(pl->alone, al, st);
        pl->nflist3 = int64_t(fl.size());
        fl.insert(fl.end(), fl_lane.begin(), fl_lane.end());
        pl->nflist = int64_t(fl.size());
        if (fl.empty()) fl.push_back(0);
        upload(pl->flist, fl, st);
        upload(pl->crange, cr, st);
    }
    pl->slab_total = slab_off;
    pl->fold_total = int64_t(fold_h.size());
    upload(pl->segs, pl->segs_h, st);
    upload(pl->fold, fold_h, st);
    std::vector<int64_t> sb_h(pl->segs_h.size());
    for (size_t s = 0; s < sb_h.size(); ++s)
        sb_h[s] = pl->segs_h[s].off - int64_t(pl->segs_h[s].z0) * pl->wins_h[pl->segs_h[s].win].lanes;
    upload(pl->sbase, sb_h, st);
    upload(pl->wins_d, pl->wins_h, st);

    // 7. matvec scratch
    pl->vs.alloc(size_t(N) * P + 2);  // two padding entries for the paired LDS staging
    pl->fs.alloc(size_t(N) * P);
    int64_t tgt_total = pl->grid_total;  // fold target-major buffer: cells x footprint positions
    {
        int64_t off = 0;
        for (int l = 0; l < P; ++l) {
            WinDev& wd = pl->wins_h[l];
            wd.tgt_off = off;
            off += int64_t(wd.E[0]) * wd.E[1] * wd.E[2] * wd.lanes;
        }
        tgt_total = std::max(tgt_total, off);
        pl->tgt_total = tgt_total;
        ANV_HIP(hipMemcpyAsync(pl->wins_d.p, pl->wins_h.data(), pl->wins_h.size() * sizeof(WinDev),
                               hipMemcpyHostToDevice, st));
    }
    if (pl->precision == ANOVA_PREC_FP64) {
        pl->g64.alloc(pl->grid_total);
        pl->h64.alloc(pl->grid_total);
        pl->c64a.alloc(tgt_total);
        pl->c64b.alloc(pl->grid_total);
        pl->slab64.alloc(pl->slab_total);
    } else {
        pl->g32.alloc(pl->grid_total);
        pl->h32.alloc(pl->grid_total);
        pl->c32a.alloc(tgt_total);
        pl->c32b.alloc(pl->grid_total);
        pl->slab32.alloc(pl->slab_total);
    }
    ANV_HIP(hipStreamSynchronize(st));
    return pl.release();
}

}  // namespace anv
