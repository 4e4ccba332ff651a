// Split-BF16 MFMA contractions (placeholder until the kernels land).
#include "mpg_internal.h"

namespace mpg {
hipError_t gemm1_bf16(const Plan &, int, const void *, int) { return hipErrorNotSupported; }
hipError_t gemm2_bf16(const Plan &, int, void *, int) { return hipErrorNotSupported; }
}  // namespace mpg
