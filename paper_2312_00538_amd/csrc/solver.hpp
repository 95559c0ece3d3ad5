// Low-rank factors, preconditioned MINRES and the interior point method.
#pragma once
#include "plan.hpp"

namespace anv {

int ipm_solve(Plan& pl, const double* labels, double C, const anova_ipm_opts& o, double* alpha,
              double* lambda, anova_ipm_stats* stats, hipStream_t st);

// returns the rank used
int pivoted_cholesky(Plan& pl, int rank, double err_tol, double* L, int64_t ldl, int64_t* piv,
                     hipStream_t st);

void nystrom_factor(Plan& pl, const double* G, int k, int64_t ldg, double* Zt, int64_t ldz,
                    hipStream_t st);

}  // namespace anv
