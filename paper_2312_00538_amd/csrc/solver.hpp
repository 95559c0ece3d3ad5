// Low-rank factors, preconditioned MINRES and the interior point method.
#pragma once
#include <functional>

#include "plan.hpp"

namespace anv {

// y = K x of one vector on a stream; replaces the plan's own matvec inside a
// solve (shared launches of several solves)
using MatvecHook = std::function<void(const double* x, double* y, hipStream_t st)>;

// Low-rank factor Z^T (N x rank, column-major) of the kernel matrix, which the
// solves of one plan with different C share: it depends on K only.
struct LowRankFactor {
    int precond = ANOVA_PRECOND_NONE;
    int rank = 0;             // columns used
    DevBuf<double> Z;
    DevBuf<float> Z32;        // FP32 copy for the N x k products (anova_ipm_opts.factor_fp32)
    double t_setup_ms = 0.0;
};

// Builds the preconditioner factor that o.precond, o.rank, o.err_tol and
// o.seed ask for (nothing for ANOVA_PRECOND_NONE).
void build_low_rank(Plan& pl, const anova_ipm_opts& o, LowRankFactor& f, hipStream_t st);

// Algorithm 1. `factor` (may be NULL) is a factor built by build_low_rank with
// the same preconditioner options; without it the solve builds its own.
// `hook` (may be NULL) performs the kernel matvecs of the iteration.
int ipm_solve(Plan& pl, const double* labels, double C, const anova_ipm_opts& o, double* alpha,
              double* lambda, anova_ipm_stats* stats, hipStream_t st, const LowRankFactor* factor = nullptr,
              const MatvecHook* hook = nullptr);

// out = (Theta + Y Z Z^T Y)^{-1} r through the capacitance refresh and the
// Woodbury passes of the IPM's preconditioner (Z: N x k, column j at Z + j*ldz;
// y NULL = identity); synchronises the stream
void lowrank_apply(int64_t N, int k, const double* Z, int64_t ldz, const double* theta, const double* y,
                   const double* r, bool fp32_products, double* out, hipStream_t st);

// returns the rank used
// uniforms: NULL for the greedy rule (Algorithm 2), else one value in [0, 1)
// per step for randomly pivoted Cholesky
int pivoted_cholesky(Plan& pl, int rank, double err_tol, double* L, int64_t ldl, int64_t* piv,
                     hipStream_t st, const double* uniforms = nullptr);

void nystrom_factor(Plan& pl, const double* G, int k, int64_t ldg, double* Zt, int64_t ldz,
                    hipStream_t st);

// random Fourier features of the plan's kernel: Z^T (N x k, column j at Z + j*ldz),
// features split over the windows as evenly as possible (earlier windows take
// the remainder); w host k x 3 (the window's coordinates in order), b host k
void rff_factor(Plan& pl, int k, const double* w, const double* b, double* Z, int64_t ldz, hipStream_t st);

// f = K(Xnew, X) (y * alpha) - lambda through one plan over both point sets
void decision_function(const double* X, int64_t N, int64_t ldx, const double* Xnew, int64_t M, int64_t ldn,
                       int32_t d, const int32_t* windows, int32_t P, const double* sigma, const double* eta,
                       const anova_opts* opts, const double* labels, const double* alpha, double lambda, double* f,
                       hipStream_t st);

}  // namespace anv
