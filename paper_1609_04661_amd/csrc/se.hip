// Scalar state evolution of D-GAMP-CT (Sec. 4.4, eqs. SEasym and
// SE_matches, the error function E_in and the sensitivity function A_in),
// evaluated on the actual phantom with the iteration's own kernels.
//
// Per iteration t (all scalars in FP64 device memory, no host sync):
//   tau_p = fro2 tau_x / M
//   output side, matched channel: P = z + sqrt(tau_p) n (n a standard-normal
//     field), tau_s = sum_i (1 - Var[z_i | P_i, y_i, tau_p] / tau_p) / (M tau_p)
//     (= -E[d g_out / dp]), damped by eta_s from t = 1; tau_r = N / (fro2 tau_s)
//   input side, xi_r = tau_r: R = x + sqrt(tau_r) v (v standard normal),
//     D(R) and the one-probe Monte-Carlo divergence (eq. MC_SURE) at R,
//     E_in = ||D(R) - x||^2 / N (the predicted MSE of the next iterate),
//     tau_x = tau_r div (A_in; div <= 0 gives 1e-12 tau_r), damped by eta_x
// z = A mu_true, x = V mu_true and the two noise fields are inputs.
#include <cmath>

#include "dg_internal.h"

namespace dg {

dg_status check_denoise_params(const dg_plan* p, int kind, const void* params);
dg_status launch_denoiser(const dg_plan* p, int kind, const void* params, const float* r,
                          const double* tau_r, const double* eps, uint64_t seed, int iter,
                          float* x_den, float* x_pert, hipStream_t st, const EpsFinish* ef,
                          const DivFuse* df);
dg_status launch_div(const dg_plan* p, const float* xden, const float* xpert, float* x,
                     const double* eps, double* div_out, double* scal, int mode, uint64_t seed,
                     int iter, double eta_x, int t, double* partials, hipStream_t st);
dg_status cnn_check_params(const dg_plan* p, const void* params);
dg_status cnn_launch_denoise(const dg_plan* p, const void* params, const float* r,
                             const double* eps, uint64_t seed, int iter, float* x_den,
                             float* x_pert, double* div_dot_out, hipStream_t st);

static constexpr int kSeBlock = 256;
static constexpr int kSeMaxBlocks = 1024;

struct SeArgs {
  int64_t M, N;
  const float* z;
  const float* x;
  const float* y;
  const float* n;
  const float* v;
  float* R;
  const float* xden;
  double* scal;
  double* dpart;
  float* fpart;
  double i0, fro2, eta_s, eta_x;
  int mode, nblk_out, nblk_in;
};

// Output side: per-block partials of sum(1 - Var/tau_p) at P = z + sqrt(tau_p) n.
__global__ void __launch_bounds__(kSeBlock) se_out_kernel(SeArgs A) {
  __shared__ double red[kSeBlock / 64];
  if (A.scal[DG_S_STATUS] != 0.0) return;
  const double tau_p_d = A.fro2 * A.scal[DG_S_TAU_X] / (double)A.M;
  const float tau_p = (float)tau_p_d, sq = (float)sqrt(tau_p_d);
  const float ln_i0 = (float)log(A.i0);
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * kSeBlock + threadIdx.x; k < A.M;
       k += (int64_t)gridDim.x * kSeBlock) {
    const float P = __fmaf_rn(sq, A.n[k], A.z[k]);
    acc += (double)poisson_channel(P, A.y[k], tau_p, ln_i0, A.mode).one_minus_v;
  }
  const double bs = block_sum(acc, red);
  if (threadIdx.x == 0) A.dpart[blockIdx.x] = bs;
}

__global__ void __launch_bounds__(256) se_out_finish(SeArgs A, int t) {
  __shared__ double red[4];
  if (A.scal[DG_S_STATUS] != 0.0) return;
  const double tot = finish_sum(A.dpart, A.nblk_out, red);
  if (threadIdx.x == 0) {
    double* s = A.scal;
    const double tau_p = A.fro2 * s[DG_S_TAU_X] / (double)A.M;
    double tau_s = tot / ((double)A.M * tau_p);
    if (t > 0) tau_s = A.eta_s * tau_s + (1.0 - A.eta_s) * s[DG_S_TAU_S];
    const double tau_r = (double)A.N / (A.fro2 * tau_s);
    s[DG_S_TAU_P] = tau_p;
    s[DG_S_TAU_S] = tau_s;
    s[DG_S_TAU_R] = tau_r;
    if (!(tau_s > 0.0) || !isfinite(tau_s) || !(tau_r > 0.0) || !isfinite(tau_r))
      s[DG_S_STATUS] = (double)(t + 1);
  }
}

// Input side: R = x + sqrt(tau_r) v and per-block max |R| (for the probe step).
__global__ void __launch_bounds__(kSeBlock) se_in_kernel(SeArgs A) {
  __shared__ float red[kSeBlock / 64];
  const bool live = A.scal[DG_S_STATUS] == 0.0;
  const float sq = live ? (float)sqrt(A.scal[DG_S_TAU_R]) : 0.0f;
  float m = 0.0f;
  for (int64_t k = (int64_t)blockIdx.x * kSeBlock + threadIdx.x; k < A.N;
       k += (int64_t)gridDim.x * kSeBlock) {
    const float r = __fmaf_rn(sq, A.v[k], A.x[k]);
    A.R[k] = r;
    m = fmaxf(m, fabsf(r));
  }
  const float bm = block_max(m, red);
  if (threadIdx.x == 0) A.fpart[blockIdx.x] = bm;
}

__global__ void __launch_bounds__(256) se_eps(SeArgs A, double eps_rel) {
  __shared__ float red[4];
  const float m = finish_max(A.fpart, A.nblk_in, red);
  if (threadIdx.x == 0) A.scal[DG_S_EPS] = fmax(eps_rel * (double)m, 1e-12);
}

// E_in partials: sum (D(R) - x)^2 per block.
__global__ void __launch_bounds__(kSeBlock) se_mse_kernel(SeArgs A) {
  __shared__ double red[kSeBlock / 64];
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * kSeBlock + threadIdx.x; k < A.N;
       k += (int64_t)gridDim.x * kSeBlock) {
    const double d = (double)A.xden[k] - (double)A.x[k];
    acc += d * d;
  }
  const double bs = block_sum(acc, red);
  if (threadIdx.x == 0) A.dpart[blockIdx.x] = bs;
}

// E_in, tau_x (A_in) and the log record of iteration t.
__global__ void __launch_bounds__(256) se_in_finish(SeArgs A, int t, double* log) {
  __shared__ double red[4];
  const double tot = finish_sum(A.dpart, A.nblk_in, red);
  if (threadIdx.x != 0) return;
  double* s = A.scal;
  double mse = 0.0;
  if (s[DG_S_STATUS] == 0.0) {
    mse = tot / (double)A.N;
    const double div = s[DG_S_DIV];
    const double tau_r = s[DG_S_TAU_R];
    double tau_x = div > 0.0 ? tau_r * div : 1e-12 * tau_r;
    if (!(div > 0.0)) s[DG_S_CLAMPS] += 1.0;
    if (t > 0) tau_x = A.eta_x * tau_x + (1.0 - A.eta_x) * s[DG_S_TAU_X];
    s[DG_S_TAU_X] = tau_x;
    if (!isfinite(div) || !(tau_x > 0.0) || !isfinite(tau_x) || !isfinite(mse))
      s[DG_S_STATUS] = (double)(t + 1);
  }
  if (log) {
    double* L = log + (size_t)t * DG_LOG_STRIDE;
    L[0] = s[DG_S_TAU_P];
    L[1] = s[DG_S_TAU_S];
    L[2] = s[DG_S_TAU_R];
    L[3] = s[DG_S_DIV];
    L[4] = s[DG_S_TAU_X];
    L[DG_SE_LOG_MSE] = mse;
    L[6] = s[DG_S_STATUS];
    L[7] = s[DG_S_CLAMPS];
  }
}

__global__ void se_init(double* scal, double tau_x0) {
  const int k = threadIdx.x;
  if (k < DG_NSCAL) scal[k] = (k == DG_S_TAU_X) ? tau_x0 : 0.0;
}

struct SeWork {
  double* scal;
  double* dpart;
  float* fpart;
  float *R, *xden, *xpert;
  double* div_part;
};

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t se_work_layout(const dg_plan* p, void* base, SeWork* w) {
  char* c = (char*)base;
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = c ? c + off : nullptr;
    off += a256(b);
    return q;
  };
  SeWork t;
  t.scal = (double*)take(sizeof(double) * DG_NSCAL);
  t.dpart = (double*)take(sizeof(double) * kSeMaxBlocks);
  t.fpart = (float*)take(sizeof(float) * kSeMaxBlocks);
  t.div_part = (double*)take(sizeof(double) * kSeMaxBlocks);
  const size_t nb = sizeof(float) * (size_t)p->N;
  t.R = (float*)take(nb);
  t.xden = (float*)take(nb);
  t.xpert = (float*)take(nb);
  if (w) *w = t;
  return off;
}

size_t se_work_bytes(const dg_plan* p) { return se_work_layout(p, nullptr, nullptr); }

}  // namespace dg

using namespace dg;

extern "C" dg_status dgamp_state_evolution(const dg_plan* p, const float* z, const float* x,
                                           const float* y, const float* n, const float* v,
                                           const dgamp_opts* o, double tau_x0, double* se_log,
                                           double* scal_out, void* work, void* stream) {
  DG_ARG_CHECK(p && z && x && y && n && v && o && work, "dgamp_state_evolution: null argument");
  DG_ARG_CHECK(o->n_iter >= 0 && o->n_iter <= 100000, "dgamp_state_evolution: bad n_iter");
  DG_ARG_CHECK(o->fro2 > 0 && std::isfinite(o->fro2), "dgamp_state_evolution: fro2 must be > 0");
  DG_ARG_CHECK(o->i0 > 0 && std::isfinite(o->i0), "dgamp_state_evolution: i0 must be > 0");
  DG_ARG_CHECK(o->eps_rel > 0 && std::isfinite(o->eps_rel),
               "dgamp_state_evolution: eps_rel must be > 0");
  DG_ARG_CHECK(o->eta_x > 0 && o->eta_x <= 1 && o->eta_s > 0 && o->eta_s <= 1,
               "dgamp_state_evolution: damping factors must be in (0, 1]");
  DG_ARG_CHECK(o->channel_mode == DG_CHANNEL_LAPLACE || o->channel_mode == DG_CHANNEL_MODE_ONLY,
               "dgamp_state_evolution: unknown channel mode");
  DG_ARG_CHECK(tau_x0 > 0 && std::isfinite(tau_x0), "dgamp_state_evolution: tau_x0 must be > 0");
  DG_ARG_CHECK(o->phase_events == nullptr, "dgamp_state_evolution: phase events not supported");
  dg_status rc = (o->den_kind == DG_DEN_CNN) ? cnn_check_params(p, o->den_params)
                                             : check_denoise_params(p, o->den_kind, o->den_params);
  if (rc != DG_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  SeWork w;
  se_work_layout(p, work, &w);
  const unsigned int go = grid_for(p->M, kSeBlock, kSeMaxBlocks);
  const unsigned int gi = grid_for(p->N, kSeBlock, kSeMaxBlocks);
  SeArgs A{p->M,   p->N,   z,      x,      y,      n,      v,         w.R,       w.xden,
           w.scal, w.dpart, w.fpart, o->i0, o->fro2, o->eta_s, o->eta_x, o->channel_mode,
           (int)go, (int)gi};
  hipLaunchKernelGGL(se_init, dim3(1), dim3(64), 0, st, w.scal, tau_x0);
  DG_LAUNCH_CHECK("se_init");
  for (int t = 0; t < o->n_iter; ++t) {
    hipLaunchKernelGGL(se_out_kernel, dim3(go), dim3(kSeBlock), 0, st, A);
    DG_LAUNCH_CHECK("se_out_kernel");
    hipLaunchKernelGGL(se_out_finish, dim3(1), dim3(256), 0, st, A, t);
    DG_LAUNCH_CHECK("se_out_finish");
    hipLaunchKernelGGL(se_in_kernel, dim3(gi), dim3(kSeBlock), 0, st, A);
    DG_LAUNCH_CHECK("se_in_kernel");
    hipLaunchKernelGGL(se_eps, dim3(1), dim3(256), 0, st, A, o->eps_rel);
    DG_LAUNCH_CHECK("se_eps");
    const double* tau_r = w.scal + DG_S_TAU_R;
    const double* eps = w.scal + DG_S_EPS;
    if (o->den_kind == DG_DEN_CNN)
      rc = cnn_launch_denoise(p, o->den_params, w.R, eps, o->probe_seed, t, w.xden, w.xpert,
                              nullptr, st);
    else
      rc = launch_denoiser(p, o->den_kind, o->den_params, w.R, tau_r, eps, o->probe_seed, t,
                           w.xden, w.xpert, st, nullptr, nullptr);
    if (rc != DG_OK) return rc;
    if ((rc = launch_div(p, w.xden, w.xpert, nullptr, eps, w.scal + DG_S_DIV, nullptr, 0,
                         o->probe_seed, t, 1.0, 0, w.div_part, st)) != DG_OK)
      return rc;
    hipLaunchKernelGGL(se_mse_kernel, dim3(gi), dim3(kSeBlock), 0, st, A);
    DG_LAUNCH_CHECK("se_mse_kernel");
    hipLaunchKernelGGL(se_in_finish, dim3(1), dim3(256), 0, st, A, t, se_log);
    DG_LAUNCH_CHECK("se_in_finish");
  }
  if (scal_out) DG_HIP(hipMemcpyAsync(scal_out, w.scal, sizeof(double) * DG_NSCAL,
                                      hipMemcpyDeviceToDevice, st));
  return DG_OK;
}
