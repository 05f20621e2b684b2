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

struct ChanOut {
  float s;
  float one_minus_v;  // 1 - Var/tau_p
};

__device__ __forceinline__ ChanOut poisson_channel(float p, float y, float tau_p, float ln_i0,
                                                   int mode) {
  const float ty = tau_p * y;
  const float ln_tp = logf(tau_p);
  const float C = ln_i0 - p;  // F(delta) = delta + ln w - ln tau_p - C
  // starting point: w0 ~ W0(e^xi), xi = ln(tau_p I0) + tau_p y - p
  const float xi = ln_tp + C + ty;
  float w0;
  if (xi > 1.0f) {
    const float lx = logf(xi);
    w0 = xi - lx + lx / xi;
  } else {
    const float e = expf(fmaxf(xi, -80.0f));
    w0 = e / (1.0f + e) * (1.0f + 0.5f * e / (1.0f + e));
  }
  float delta = w0 - ty;
  // Halley on F with F' = (w+1)/w and F'' = -1/w^2, written without 1/w so
  // that no term overflows for small w; Newton when the Halley denominator
  // is not safely positive.
#pragma unroll
  for (int it = 0; it < 5; ++it) {
    const float w = fmaxf(delta + ty, 1e-30f);
    const float F = delta + logf(w) - ln_tp - C;
    const float w1 = w + 1.0f;
    const float den = 2.0f * w1 * w1 + F;
    delta -= (den > w1 * w1) ? 2.0f * F * w1 * w / den : F * w / w1;
  }
  const float w = fmaxf(delta + ty, 1e-30f);
  const float u = 1.0f / (1.0f + w);
  ChanOut o;
  if (mode == DG_CHANNEL_MODE_ONLY) {
    o.s = delta / tau_p;
    o.one_minus_v = 1.0f - u;
    return o;
  }
  const float u2 = u * u;
  o.s = delta / tau_p + 0.5f * w * u2;
  float v = u - 0.5f * w * tau_p * u2 * u + w * w * tau_p * u2 * u2;
  v = fminf(fmaxf(v, 0.0f), 1.0f);
  o.one_minus_v = 1.0f - v;
  return o;
}

// Fused form used inside the iteration:
//   tau_p = fro2 tau_x / M, p = z - tau_p s_prev, s = channel(p),
//   s <- eta_s s + (1 - eta_s) s_prev  (t > 0), and the last block finishes
//   tau_s (damped likewise) and tau_r = N / (fro2 tau_s).
// Standalone form: p given, tau_p from a device scalar, writes s and tau_s.
template <bool kFused>
__device__ void channel_body(const ChanArgs& A, int blk, int mode, double eta_s, int onsager,
                             int t, double* red) {
  double tau_p_d;
  if (kFused) {
    if (A.scal[DG_S_STATUS] != 0.0) return;
    tau_p_d = A.fro2 * A.scal[DG_S_TAU_X] / (double)A.M;
  } else {
    tau_p_d = *A.tau_p_ptr;
  }
  const float tau_p = (float)tau_p_d;
  const float ln_i0 = (float)log(A.i0);
  const float eta = (float)eta_s;
  double acc = 0.0;
  for (int64_t k = (int64_t)blk * kChanBlock + threadIdx.x; k < A.M;
       k += (int64_t)A.nblk * kChanBlock) {
    float p = A.zp[k];
    float s_prev = 0.0f;
    if (kFused) {
      s_prev = A.s_io[k];
      if (onsager) p = __fmaf_rn(-tau_p, s_prev, p);
    }
    ChanOut o = poisson_channel(p, A.y[k], tau_p, ln_i0, mode);
    float s = o.s;
    if (kFused) {
      if (t > 0) s = __fmaf_rn(eta, s, (1.0f - eta) * s_prev);
      A.s_io[k] = s;
    } else {
      A.s_out[k] = s;
    }
    acc += (double)o.one_minus_v;
  }
  double bs = block_sum(acc, red);
  if (threadIdx.x == 0) A.partials[blk] = bs;
}

template <bool kFused>
__global__ void __launch_bounds__(kChanBlock)
channel_kernel(ChanArgs A, int mode, double eta_s, int onsager, int t) {
  __shared__ double red[kChanBlock / 64];
  channel_body<kFused>(A, blockIdx.x, mode, eta_s, onsager, t, red);
}
__global__ void __launch_bounds__(kChanBlock)
channel_batch(const ChanArgs* __restrict__ T, const int* __restrict__ prefix, int n, int mode,
              double eta_s, int onsager, int t) {
  __shared__ double red[kChanBlock / 64];
  const int s = slice_of(prefix, n, blockIdx.x);
  channel_body<true>(T[s], blockIdx.x - prefix[s], mode, eta_s, onsager, t, red);
}
template <bool kFused>
__global__ void __launch_bounds__(256) channel_finish(ChanArgs A, double eta_s, int t) {
  __shared__ double red[4];
  channel_finish_body<kFused>(A, eta_s, t, red);
}
__global__ void __launch_bounds__(256)
channel_finish_batch(const ChanArgs* __restrict__ T, double eta_s, int t) {
  __shared__ double red[4];
  channel_finish_body<true>(T[blockIdx.x], eta_s, t, red);
}

unsigned int channel_grid(int64_t M) { return grid_for(M, kChanBlock, kChanMaxBlocks); }

// Inside the iteration.  With finish = 0 the caller finishes the channel
// later (channel_finish_body on *out_args); the arguments are returned in
// out_args either way.
dg_status launch_channel_fused(int64_t M, const float* z, const float* y, float* s, double* scal,
                               double i0, int mode, double fro2, double N, double eta_s,
                               int onsager, int t, double* partials, int finish,
                               ChanArgs* out_args, hipStream_t st) {
  const unsigned int g = channel_grid(M);
  ChanArgs A{M, z, y, s, nullptr, nullptr, scal, nullptr, i0, fro2, N, partials, (int)g};
  if (out_args) *out_args = A;
  hipLaunchKernelGGL(channel_kernel<true>, dim3(g), dim3(kChanBlock), 0, st, A, mode, eta_s,
                     onsager, t);
  DG_LAUNCH_CHECK("channel_kernel<fused>");
  if (finish) {
    hipLaunchKernelGGL(channel_finish<true>, dim3(1), dim3(256), 0, st, A, eta_s, t);
    DG_LAUNCH_CHECK("channel_finish<fused>");
  }
  return DG_OK;
}

// finish = 0: the finish runs later, inside the first row pass of the
// next preconditioner application.
dg_status launch_channel_batch(const ChanArgs* T, const int* prefix, int n, int total, int mode,
                               double eta_s, int onsager, int t, int finish, hipStream_t st) {
  hipLaunchKernelGGL(channel_batch, dim3(total), dim3(kChanBlock), 0, st, T, prefix, n, mode, eta_s,
                     onsager, t);
  DG_LAUNCH_CHECK("channel_batch");
  if (finish) {
    hipLaunchKernelGGL(channel_finish_batch, dim3(n), dim3(256), 0, st, T, eta_s, t);
    DG_LAUNCH_CHECK("channel_finish_batch");
  }
  return DG_OK;
}

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
  hipLaunchKernelGGL(channel_kernel<false>, dim3(g), dim3(kChanBlock), 0, st, A, mode, 1.0, 0, 0);
  DG_LAUNCH_CHECK("channel_kernel");
  hipLaunchKernelGGL(channel_finish<false>, dim3(1), dim3(256), 0, st, A, 1.0, 0);
  DG_LAUNCH_CHECK("channel_finish");
  return DG_OK;
}
