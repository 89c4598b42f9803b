// Learned warm start: MLP 12 -> 64 -> 64 -> 64 -> 3 (ReLU) on BF16 MFMA tiles.
#include <hip/hip_runtime.h>

#include "nsn_layout.h"

namespace nsn {
hipError_t launch_warm_mlp(const DevScene &, hipStream_t) { return hipErrorNotSupported; }
}  // namespace nsn

extern "C" {
nsn_status nsn_mlp_forward(const float *, const float *, float *, int64_t, void *) { return NSN_EUNSUPPORTED; }
size_t nsn_mlp_scratch_bytes(int64_t) { return 0; }
nsn_status nsn_mlp_loss_grad(const float *, const float *, const float *, int64_t, float *, float *, void *, void *) {
  return NSN_EUNSUPPORTED;
}
nsn_status nsn_mlp_adam(float *, const float *, float *, float *, int64_t, float, float, float, float, int32_t, void *) {
  return NSN_EUNSUPPORTED;
}
}
