// Residual CNN denoiser (placeholder until the MFMA kernels land).
#include "dg_internal.h"

namespace dg {

dg_status cnn_check_params(const dg_plan* p, const void* params) {
  (void)p;
  (void)params;
  set_error("denoise: CNN denoiser not available in this build");
  return DG_ERR_UNSUPPORTED;
}

dg_status cnn_launch_denoise(const dg_plan*, const void*, const float*, const double*, uint64_t,
                             int, float*, float*, double*, hipStream_t) {
  set_error("denoise: CNN denoiser not available in this build");
  return DG_ERR_UNSUPPORTED;
}

}  // namespace dg
