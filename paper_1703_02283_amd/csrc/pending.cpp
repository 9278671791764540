// Entry points declared in include/ipr.h whose kernels are not in this build
// yet: they fail with IPR_EARG and a message instead of computing anything.
#include <hip/hip_runtime.h>

#include "../../include/ipr.h"
#include "ipr_host.h"

using namespace ipr;

extern "C" {

int ipr_features(const double*, const int64_t*, const int*, const int*, int, float*, void*, size_t,
                 hipStream_t) {
  return fail(IPR_EARG, "ipr_features is not available in this build");
}
int ipr_mlp_forward(const float*, const float*, float*, int, hipStream_t) {
  return fail(IPR_EARG, "ipr_mlp_forward is not available in this build");
}
int ipr_mlp_train_step(float*, float*, float*, float*, const float*, const float*, int, int, float,
                       float*, void*, size_t, hipStream_t) {
  return fail(IPR_EARG, "ipr_mlp_train_step is not available in this build");
}
size_t ipr_mlp_workspace(int) { return 0; }
}
