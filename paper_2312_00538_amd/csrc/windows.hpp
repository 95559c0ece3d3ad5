// Windows of features by mutual-information ranking (see windows.hip).
#pragma once
#include "common.hpp"

namespace anv {

void mi_windows(const double* X, int64_t N, int32_t d, int64_t ldx, const double* labels, int32_t bins, int32_t P,
                int32_t* windows, double* mi, hipStream_t st);

}  // namespace anv
