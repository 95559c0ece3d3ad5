// Autotuner of the fast-summation options for one data set: bandwidth, cutoff,
// precision and work-item size (Section 3 leaves N and m to the user; the
// error of the NFFT-based sum falls with both, its cost grows with both).
//
// Every candidate plan is built, its matvec of a seeded random block is
// compared with that of a high-accuracy FP64 reference plan (bandwidth 64,
// cutoff 4), and the candidates within the target error are timed with HIP
// events on the caller's stream for the caller's number of right-hand sides.
// The fastest one wins; a second pass varies its work-item size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "plan.hpp"
#include "tune.hpp"

namespace anv {

namespace {

constexpr int kT = 256;
inline unsigned nblk(int64_t n) { return unsigned(std::max<int64_t>(1, (n + kT - 1) / kT)); }

// splitmix64 (Steele, Lea and Flood 2014) of a counter
__device__ inline uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// standard normal variates by the Box-Muller transform of two counter-based uniforms
__global__ void k_normal(double* __restrict__ x, int64_t n, uint64_t seed) {
    const int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i >= n) return;
    const uint64_t a = splitmix64(seed ^ (2 * uint64_t(i))), b = splitmix64(seed ^ (2 * uint64_t(i) + 1));
    const double u1 = (double(a >> 11) + 1.0) * 0x1.0p-53;  // (0, 1]
    const double u2 = double(b >> 11) * 0x1.0p-53;          // [0, 1)
    x[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// per-block partial sums of (a - b)^2 and b^2
__global__ void k_err_parts(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                            double* __restrict__ part) {
    __shared__ double s0[kT], s1[kT];
    double e = 0.0, r = 0.0;
    for (int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kT) {
        const double d = a[i] - b[i];
        e += d * d;
        r += b[i] * b[i];
    }
    s0[threadIdx.x] = e;
    s1[threadIdx.x] = r;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) {
            s0[threadIdx.x] += s0[threadIdx.x + s];
            s1[threadIdx.x] += s1[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

struct Job {
    anova_opts o;
    double err = -1.0, ms = -1.0;
};

}  // namespace

int autotune(const double* X, int64_t N, int32_t d, int64_t ldx, const int32_t* windows, int32_t P,
             const double* sigma, const double* eta, const anova_tune_opts& t, hipStream_t st, anova_opts* best,
             anova_tune_candidate* cands, int32_t max_cands, int32_t* n_cands) {
    ANV_CHECK(best != nullptr, "NULL output");
    ANV_CHECK(t.rhs >= 1 && t.rhs <= 64, "rhs must be in [1, 64]");
    ANV_CHECK(std::isfinite(t.target_rel_err) && t.target_rel_err > 0.0, "target_rel_err must be > 0");
    ANV_CHECK((t.precisions & 3) != 0, "no precision selected");
    ANV_CHECK(t.reps >= 1 && t.reps <= 100, "reps must be in [1, 100]");
    const int R = t.rhs;
    DevBuf<double> x, yref, y, part;
    x.alloc(size_t(N) * R);
    yref.alloc(size_t(N) * R);
    y.alloc(size_t(N) * R);
    const unsigned nb = std::min<unsigned>(256, nblk(N * R));
    part.alloc(size_t(nb) * 2);
    hipLaunchKernelGGL(k_normal, dim3(nblk(N * R)), dim3(kT), 0, st, x.p, N * R, t.seed);

    auto build = [&](const anova_opts& o) {
        return std::unique_ptr<Plan>(create_plan(X, N, d, ldx, windows, P, sigma, eta, &o, st));
    };
    // the reference: FP64, bandwidth 64 (32 if the occupied box does not fit), cutoff 4
    anova_opts ro;
    anova_opts_default(&ro);
    ro.batch_min_rhs = -1;
    std::unique_ptr<Plan> ref;
    for (int nbw : {64, 32}) {
        ro.n_bw = nbw;
        try {
            ref = build(ro);
            break;
        } catch (const Error&) {
            if (nbw == 32) throw;
        }
    }
    enqueue_matvec(*ref, x.p, R, N, yref.p, N, st);
    ref.reset();

    std::vector<double> hp(size_t(nb) * 2);
    auto rel_err = [&]() {
        hipLaunchKernelGGL(k_err_parts, dim3(nb), dim3(kT), 0, st, y.p, yref.p, N * R, part.p);
        ANV_HIP(hipMemcpyAsync(hp.data(), part.p, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        ANV_HIP(hipStreamSynchronize(st));
        double e = 0.0, r = 0.0;
        for (unsigned b = 0; b < nb; ++b) {
            e += hp[2 * b];
            r += hp[2 * b + 1];
        }
        return r > 0.0 ? std::sqrt(e / r) : 0.0;
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ANV_HIP(hipEventCreate(&e0));
    ANV_HIP(hipEventCreate(&e1));
    struct EvFree {
        hipEvent_t a, b;
        ~EvFree() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev_guard{e0, e1};
    auto time_ms = [&](Plan& pl) {
        enqueue_matvec(pl, x.p, R, N, y.p, N, st);  // warm-up (allocates the batched buffers)
        ANV_HIP(hipEventRecord(e0, st));
        for (int i = 0; i < t.reps; ++i) enqueue_matvec(pl, x.p, R, N, y.p, N, st);
        ANV_HIP(hipEventRecord(e1, st));
        ANV_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        ANV_HIP(hipEventElapsedTime(&ms, e0, e1));
        return double(ms) / t.reps;
    };
    // one candidate: build, check the error, time it if admissible
    auto evaluate = [&](Job& j) {
        std::unique_ptr<Plan> pl;
        try {
            pl = build(j.o);
        } catch (const Error& e) {
            if (e.code != ANOVA_INVALID_ARG) throw;  // a size this data set cannot use
            return;
        }
        enqueue_matvec(*pl, x.p, R, N, y.p, N, st);
        j.err = rel_err();
        if (j.err <= t.target_rel_err) j.ms = time_ms(*pl);
    };

    std::vector<Job> jobs;
    for (int prec : {ANOVA_PREC_MIXED, ANOVA_PREC_FP64}) {
        if (!(t.precisions & (prec == ANOVA_PREC_FP64 ? 1 : 2))) continue;
        for (int m : {2, 3, 4})
            for (int nbw : {16, 24, 32, 48, 64}) {
                Job j;
                anova_opts_default(&j.o);
                j.o.precision = prec;
                j.o.cutoff_m = m;
                j.o.n_bw = nbw;
                jobs.push_back(j);
            }
    }
    int win = -1;
    for (size_t i = 0; i < jobs.size(); ++i) {
        evaluate(jobs[i]);
        if (jobs[i].ms >= 0.0 && (win < 0 || jobs[i].ms < jobs[size_t(win)].ms)) win = int(i);
    }
    if (win >= 0) {
        // second pass: the work-item size of the winner (points per spreading item)
        const anova_opts w = jobs[size_t(win)].o;
        for (int sp : {384, 1536}) {
            Job j;
            j.o = w;
            j.o.seg_points = sp;
            jobs.push_back(j);
            evaluate(jobs.back());
            if (jobs.back().ms >= 0.0 && jobs.back().ms < jobs[size_t(win)].ms) win = int(jobs.size() - 1);
        }
    }
    if (n_cands) *n_cands = int32_t(jobs.size());
    if (cands) {
        for (size_t i = 0; i < jobs.size() && int32_t(i) < max_cands; ++i) {
            anova_tune_candidate& c = cands[i];
            c.n_bw = jobs[i].o.n_bw;
            c.cutoff_m = jobs[i].o.cutoff_m;
            c.precision = jobs[i].o.precision;
            c.seg_points = jobs[i].o.seg_points;
            c.rel_err = jobs[i].err;
            c.ms = jobs[i].ms;
        }
    }
    if (win < 0) throw Error(ANOVA_NOT_CONVERGED, "no candidate reaches the target error");
    *best = jobs[size_t(win)].o;
    return int(win);
}

}  // namespace anv
