// Mixed-precision evaluation (FP32 basis, split-BF16 MFMA contraction, FP64
// anchor sum).
#include "hdmr_internal.h"

using namespace hdmr;

extern "C" __attribute__((visibility("hidden"))) int hdmr_eval_mixed_impl(const hdmr_model *model, const double *points, int64_t n, double *values,
                                    hipStream_t stream) {
  (void)model; (void)points; (void)n; (void)values; (void)stream;
  return fail(HDMR_EUNSUPPORTED, "mixed precision path not built yet");
}
