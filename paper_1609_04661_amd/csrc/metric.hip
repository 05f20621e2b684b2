// Reconstruction quality on the device: PSNR of an estimate against the
// true image, as Sec. 6 reports it (peak = largest true value, MSE over all
// pixels), with FP64 accumulation.  Attenuation images are non-negative; the
// peak is taken as max(0, max ref).
#include <cmath>

#include "dg_internal.h"

namespace dg {

static constexpr int kPsnrBlocks = 1024;

__global__ void __launch_bounds__(256)
psnr_partial(const float* __restrict__ est, const float* __restrict__ ref, int64_t n,
             double* __restrict__ sq_part, float* __restrict__ max_part) {
  __shared__ double dred[4];
  __shared__ float fred[4];
  double acc = 0.0;
  float mx = 0.0f;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
    const float r = ref[k];
    const double d = (double)est[k] - (double)r;
    acc = fma(d, d, acc);
    mx = fmaxf(mx, r);
  }
  const double s = block_sum(acc, dred);
  const float m = block_max(mx, fred);
  if (threadIdx.x == 0) {
    sq_part[blockIdx.x] = s;
    max_part[blockIdx.x] = m;
  }
}

__global__ void __launch_bounds__(256)
psnr_finish(const double* __restrict__ sq_part, const float* __restrict__ max_part, int nblk,
            int64_t n, double* __restrict__ out) {
  __shared__ double dred[4];
  __shared__ float fred[4];
  double s = 0.0;
  float m = 0.0f;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
    s += sq_part[k];
    m = fmaxf(m, max_part[k]);
  }
  s = block_sum(s, dred);
  m = block_max(m, fred);
  if (threadIdx.x == 0) {
    const double mse = s / (double)n;
    *out = 10.0 * log10((double)m * (double)m / mse);
  }
}

}  // namespace dg

using namespace dg;

extern "C" size_t dg_psnr_workspace_bytes(void) {
  return sizeof(double) * kPsnrBlocks + sizeof(float) * kPsnrBlocks;
}

extern "C" dg_status dg_psnr(int64_t n, const float* est, const float* ref, double* out,
                             void* work, void* stream) {
  DG_ARG_CHECK(n >= 1 && est && ref && out && work, "dg_psnr: bad argument");
  hipStream_t st = (hipStream_t)stream;
  double* sq = (double*)work;
  float* mx = (float*)(sq + kPsnrBlocks);
  const unsigned int g = grid_for(n, 256, kPsnrBlocks);
  hipLaunchKernelGGL(psnr_partial, dim3(g), dim3(256), 0, st, est, ref, n, sq, mx);
  DG_LAUNCH_CHECK("psnr_partial");
  hipLaunchKernelGGL(psnr_finish, dim3(1), dim3(256), 0, st, sq, mx, (int)g, n, out);
  DG_LAUNCH_CHECK("psnr_finish");
  return DG_OK;
}
