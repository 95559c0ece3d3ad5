// (filled in below)
#include "solver.hpp"

namespace anv {

int ipm_solve(Plan&, const double*, double, const anova_ipm_opts&, double*, double*,
              anova_ipm_stats*, hipStream_t) {
    throw Error(ANOVA_INVALID_ARG, "svm_ipm_solve: not built yet");
}
int pivoted_cholesky(Plan&, int, double, double*, int64_t, int64_t*, hipStream_t) {
    throw Error(ANOVA_INVALID_ARG, "pivoted Cholesky: not built yet");
}
void nystrom_factor(Plan&, const double*, int, int64_t, double*, int64_t, hipStream_t) {
    throw Error(ANOVA_INVALID_ARG, "Nystrom: not built yet");
}

}  // namespace anv
