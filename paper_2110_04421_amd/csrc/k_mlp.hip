// Calibration network kernels (placeholder entry points until the MFMA kernels land).
#include "abm_internal.h"

extern "C" {
int abm_mlp_workspace_size(int32_t, size_t* bytes) {
  if (bytes) *bytes = 0;
  return ABM_E_STATE;
}
int abm_mlp_forward(void*, size_t, const uint16_t*, const float*, int32_t, float*, void*) { return ABM_E_STATE; }
int abm_mlp_backward(void*, size_t, const uint16_t*, const float*, int32_t, int32_t, float*, float*, void*) {
  return ABM_E_STATE;
}
int abm_mlp_adam(float*, uint16_t*, float*, float*, const float*, float, float, float, float, int32_t, void*) {
  return ABM_E_STATE;
}
}
