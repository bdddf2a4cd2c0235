// Reduced-precision Gram forms (FP32 MFMA, split-BF16x3 MFMA).
#include "common.hpp"

size_t gram_lowp_workspace(int /*algo*/, int64_t /*n*/, int64_t /*k*/) { return 0; }

int gram_lowp(hipStream_t, int, const float*, int64_t, int64_t, int64_t, const double*, const double*, int,
              const int64_t*, double*, int64_t, void*, size_t) {
  return dopinf::fail(DOPINF_E_ARG, "reduced-precision Gram not available in this build");
}
