// BF16 and split-BF16 leaf products (placeholder until the MFMA bf16 kernel
// lands: reports the combination as unsupported).
#include "internal.h"

namespace spamm {

bool gemm_bf16_built() { return false; }

hipError_t launch_gemm_bf16(hipStream_t, int, int, const ReqDev*, const WorkUnit*, const int64_t*, int64_t, int32_t*,
                            int) {
  return hipErrorNotSupported;
}

}  // namespace spamm
