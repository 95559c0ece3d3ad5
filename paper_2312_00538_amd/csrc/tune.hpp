// Autotuner of the fast-summation options (see tune.hip).
#pragma once
#include "common.hpp"

namespace anv {

// Returns the index of the chosen candidate; throws Error(ANOVA_NOT_CONVERGED)
// when no candidate reaches the target error.
int autotune(const double* X, int64_t N, int32_t d, int64_t ldx, const int32_t* windows, int32_t P,
             const double* sigma, const double* eta, const anova_tune_opts& t, hipStream_t st, anova_opts* best,
             anova_tune_candidate* cands, int32_t max_cands, int32_t* n_cands);

}  // namespace anv
