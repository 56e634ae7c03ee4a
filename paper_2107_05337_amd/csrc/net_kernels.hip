// net_kernels.hip -- learned warm start (placeholder entry points until the network kernels land).
#include <hip/hip_runtime.h>

#include "../../include/pmgrit.h"

extern "C" {
int64_t pmgrit_net_nparams(void) { return 0; }
pmgrit_status pmgrit_net_load(pmgrit_handle*, const float*, int64_t) { return PMGRIT_E_STATE; }
pmgrit_status pmgrit_net_save(const pmgrit_handle*, float*, int64_t) { return PMGRIT_E_STATE; }
pmgrit_status pmgrit_net_forward(pmgrit_handle*, int32_t, int32_t, const float*, float*, void*) { return PMGRIT_E_STATE; }
pmgrit_status pmgrit_net_train_step(pmgrit_handle*, int32_t, int32_t, const float*, const float*, float, float*, void*) {
  return PMGRIT_E_STATE;
}
pmgrit_status pmgrit_net_grad(pmgrit_handle*, int32_t, int32_t, const float*, const float*, float*, float*, void*) {
  return PMGRIT_E_STATE;
}
}
