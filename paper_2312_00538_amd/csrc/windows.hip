// Windows of features by mutual-information ranking. Section 3 builds each
// window from the features' mutual-information scores. Here each feature's
// mutual information with the labels is estimated from a histogram of
// equal-width bins over the feature's range against the two classes; the
// features are ranked by it (largest first, ties to the lower index) and the
// windows are consecutive triples of the ranking.
//
// The GPU reduces each feature to its range and its integer histogram (the
// counts do not depend on the order of the atomic adds); the host turns the
// d x bins x 2 counts into the estimates and the ranking.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "windows.hpp"

namespace anv {

namespace {

constexpr int kT = 256;
constexpr int kMaxBins = 1024;

// part[(f * gridDim.x + b) * 3 + {0, 1, 2}] = min and max of feature f over
// block b's rows, and the number of NaN or infinite entries among them
__global__ __launch_bounds__(kT) void k_col_range(const double* __restrict__ X, int64_t N, int64_t ldx,
                                                  double* __restrict__ part) {
    const int f = blockIdx.y;
    double lo = INFINITY, hi = -INFINITY, bad = 0.0;
    for (int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x; i < N; i += int64_t(gridDim.x) * kT) {
        const double x = X[i * ldx + f];
        if (isfinite(x)) {
            lo = fmin(lo, x);
            hi = fmax(hi, x);
        } else {
            bad += 1.0;
        }
    }
    __shared__ double slo[kT], shi[kT], sbad[kT];
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) {
            slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + s]);
            shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + s]);
            sbad[threadIdx.x] += sbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t o = (int64_t(f) * gridDim.x + blockIdx.x) * 3;
        part[o] = slo[0];
        part[o + 1] = shi[0];
        part[o + 2] = sbad[0];
    }
}

// counts[(f * bins + b) * 2 + c] += number of rows with bin b of feature f and
// class c (0: label -1, 1: label +1); bin b = floor((x - lo_f) * scale_f),
// clamped to bins - 1 (scale_f = 0 for a constant feature)
#pragma clang fp contract(off)
__global__ __launch_bounds__(kT) void k_col_hist(const double* __restrict__ X, int64_t N, int64_t ldx,
                                                 const double* __restrict__ y, const double* __restrict__ lo_scale,
                                                 int bins, unsigned long long* __restrict__ counts) {
    const int f = blockIdx.y;
    __shared__ unsigned int h[2 * kMaxBins];
    for (int e = threadIdx.x; e < 2 * bins; e += kT) h[e] = 0u;
    __syncthreads();
    const double lo = lo_scale[2 * f], scale = lo_scale[2 * f + 1];
    for (int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x; i < N; i += int64_t(gridDim.x) * kT) {
        const double t = floor((X[i * ldx + f] - lo) * scale);
        const int b = t < double(bins - 1) ? int(t) : bins - 1;
        atomicAdd(&h[2 * b + (y[i] > 0.0 ? 1 : 0)], 1u);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * bins; e += kT)
        if (h[e]) atomicAdd(&counts[int64_t(f) * 2 * bins + e], (unsigned long long)h[e]);
}

}  // namespace

void mi_windows(const double* X, int64_t N, int32_t d, int64_t ldx, const double* labels, int32_t bins, int32_t P,
                int32_t* windows, double* mi, hipStream_t st) {
    ANV_CHECK(X && labels && windows, "NULL argument");
    ANV_CHECK(N >= 1 && d >= 1 && ldx >= d, "need N >= 1, d >= 1, ldx >= d");
    ANV_CHECK(bins >= 2 && bins <= kMaxBins, "bins must be in [2, 1024]");
    ANV_CHECK(P >= 1 && P <= (d + 2) / 3, "P must be in [1, ceil(d / 3)]");
    const unsigned nb = unsigned(std::min<int64_t>(256, (N + kT - 1) / kT));
    DevBuf<double> part, ls;
    DevBuf<unsigned long long> cnt;
    part.alloc(size_t(d) * nb * 3);
    ls.alloc(size_t(d) * 2);
    cnt.alloc(size_t(d) * bins * 2);
    hipLaunchKernelGGL(k_col_range, dim3(nb, unsigned(d)), dim3(kT), 0, st, X, N, ldx, part.p);
    std::vector<double> hp(size_t(d) * nb * 3), hls(size_t(d) * 2);
    ANV_HIP(hipMemcpyAsync(hp.data(), part.p, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    ANV_HIP(hipStreamSynchronize(st));
    for (int f = 0; f < d; ++f) {
        double lo = INFINITY, hi = -INFINITY, bad = 0.0;
        for (unsigned b = 0; b < nb; ++b) {
            lo = std::min(lo, hp[(size_t(f) * nb + b) * 3]);
            hi = std::max(hi, hp[(size_t(f) * nb + b) * 3 + 1]);
            bad += hp[(size_t(f) * nb + b) * 3 + 2];
        }
        ANV_CHECK(bad == 0.0, "X holds NaN or Inf");
        hls[2 * f] = lo;
        hls[2 * f + 1] = hi > lo ? double(bins) / (hi - lo) : 0.0;
    }
    ANV_HIP(hipMemcpyAsync(ls.p, hls.data(), hls.size() * sizeof(double), hipMemcpyHostToDevice, st));
    ANV_HIP(hipMemsetAsync(cnt.p, 0, cnt.bytes(), st));
    hipLaunchKernelGGL(k_col_hist, dim3(nb, unsigned(d)), dim3(kT), 0, st, X, N, ldx, labels, ls.p, bins, cnt.p);
    std::vector<unsigned long long> hc(size_t(d) * bins * 2);
    ANV_HIP(hipMemcpyAsync(hc.data(), cnt.p, hc.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    ANV_HIP(hipStreamSynchronize(st));
    // mutual information per feature: sum over n > 0 of (n / N) log(n N / (n_b n_c))
    std::vector<double> est(d);
    for (int f = 0; f < d; ++f) {
        const unsigned long long* c = hc.data() + size_t(f) * bins * 2;
        unsigned long long ncls[2] = {0, 0};
        for (int b = 0; b < bins; ++b) {
            ncls[0] += c[2 * b];
            ncls[1] += c[2 * b + 1];
        }
        const double Nt = double(ncls[0] + ncls[1]);
        double s = 0.0;
        for (int b = 0; b < bins; ++b) {
            const double nbin = double(c[2 * b] + c[2 * b + 1]);
            for (int k = 0; k < 2; ++k) {
                const double n = double(c[2 * b + k]);
                if (n > 0.0) s += (n / Nt) * std::log(n * Nt / (nbin * double(ncls[k])));
            }
        }
        est[f] = s;
    }
    std::vector<int> rank(d);
    std::iota(rank.begin(), rank.end(), 0);
    std::stable_sort(rank.begin(), rank.end(), [&](int a, int b) { return est[a] > est[b]; });
    for (int l = 0; l < P; ++l)
        for (int j = 0; j < 3; ++j) {
            const int r = 3 * l + j;
            windows[3 * l + j] = r < d ? rank[r] : -1;
        }
    if (mi) std::copy(est.begin(), est.end(), mi);
}

}  // namespace anv
