// GAMP output channel for Poisson transmission counts (Sec. 4.2 eqs.
// noise_mod / MMSEmm / post_exp, Appendix A, Algorithm 1 step 2).
//
// Per ray the posterior of z is exp(L(z)), L = -(z-p)^2/(2 tau_p) - y z - I0 e^-z.
// The mode is found in the variable delta = z0 - p, which avoids the
// cancellation of the closed form z0 = p - tau_p y + W0(...): with
// w = delta + tau_p y (= tau_p * I0 e^-z0 at the mode), delta solves
//     F(delta) = delta + ln(w / tau_p) - (ln I0 - p) = 0,
// an increasing concave equation solved by Halley steps from the log-domain
// Lambert-W starting point.  Then, with lambda = w / tau_p and
// sigma^2 = tau_p / (1 + w), the second-order Laplace (fully exponential)
// moments are
//     E[z] - p   = delta + w tau_p / (2 (1+w)^2)
//     Var/tau_p  = 1/(1+w) - w tau_p/(2 (1+w)^3) + w^2 tau_p/(1+w)^4, clamped to [0,1],
// and s = (E[z] - p)/tau_p, tau_s = sum(1 - Var/tau_p) / (M tau_p) with the
// sum in FP64 (per-block partials, finished by the last block in order).
#include <cmath>

#include "dg_internal.h"

namespace dg {

static constexpr int kChanBlock = 256;
static constexpr int kChanMaxBlocks = 1024;

// Standalone form (gamp_poisson_out): p given, tau_p from a device scalar,
// writes s and the per-block partials of sum(1 - Var/tau_p), finished into
// tau_s by channel_finish.  Inside the iteration the same per-ray math runs
// in the projector's epilogue (fused form: tau_p = fro2 tau_x / M,
// p = z - tau_p s_prev, s damped towards s_prev), and the finish (tau_s
// damped likewise, tau_r = N / (fro2 tau_s)) in the row pass of the next
// preconditioner application (a workgroup of its own beside the transforms;
// a slice's first row workgroup in batches).
__device__ void channel_body(const ChanArgs& A, int blk, int mode, double* red) {
  const float tau_p = (float)(*A.tau_p_ptr);
  const float ln_i0 = (float)log(A.i0);
  double acc = 0.0;
  for (int64_t k = (int64_t)blk * kChanBlock + threadIdx.x; k < A.M;
       k += (int64_t)A.nblk * kChanBlock) {
    const ChanOut o = poisson_channel(A.zp[k], A.y[k], tau_p, ln_i0, mode);
    A.s_out[k] = o.s;
    acc += (double)o.one_minus_v;
  }
  double bs = block_sum(acc, red);
  if (threadIdx.x == 0) A.partials[blk] = bs;
}

__global__ void __launch_bounds__(kChanBlock) channel_kernel(ChanArgs A, int mode) {
  __shared__ double red[kChanBlock / 64];
  channel_body(A, blockIdx.x, mode, red);
}
__global__ void __launch_bounds__(256) channel_finish(ChanArgs A) {
  __shared__ double red[4];
  channel_finish_body<false>(A, 1.0, 0, red);
}

unsigned int channel_grid(int64_t M) { return grid_for(M, kChanBlock, kChanMaxBlocks); }

__global__ void zero_u32(unsigned int* p, int n) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0u;
}

dg_status launch_zero_u32(unsigned int* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_u32, dim3((n + 63) / 64), dim3(64), 0, st, p, n);
  DG_LAUNCH_CHECK("zero_u32");
  return DG_OK;
}

}  // namespace dg

using namespace dg;

extern "C" size_t dg_channel_workspace_bytes(int64_t m) {
  (void)m;
  return 256 + sizeof(double) * (size_t)kChanMaxBlocks;
}

extern "C" dg_status gamp_poisson_out(int64_t m, const float* p, const float* y,
                                      const double* tau_p, double i0, int32_t mode, float* s_out,
                                      double* tau_s_out, void* work, void* stream) {
  DG_ARG_CHECK(m > 0, "gamp_poisson_out: m must be > 0");
  DG_ARG_CHECK(p && y && tau_p && s_out && tau_s_out && work, "gamp_poisson_out: null argument");
  DG_ARG_CHECK(i0 > 0 && std::isfinite(i0), "gamp_poisson_out: i0 must be > 0");
  DG_ARG_CHECK(mode == DG_CHANNEL_LAPLACE || mode == DG_CHANNEL_MODE_ONLY,
               "gamp_poisson_out: unknown mode");
  hipStream_t st = (hipStream_t)stream;
  double* partials = (double*)((char*)work + 256);
  const unsigned int g = channel_grid(m);
  ChanArgs A{m, p, y, nullptr, s_out, tau_p, nullptr, tau_s_out, i0, 0.0, 0.0, partials, (int)g};
  hipLaunchKernelGGL(channel_kernel, dim3(g), dim3(kChanBlock), 0, st, A, mode);
  DG_LAUNCH_CHECK("channel_kernel");
  hipLaunchKernelGGL(channel_finish, dim3(1), dim3(256), 0, st, A);
  DG_LAUNCH_CHECK("channel_finish");
  return DG_OK;
}
