// Proximal total-variation denoiser (the paper's second plug-in family,
// Sec. 6 "Proximal-based TV denoiser"; Sec. 4.3 treats D as a black box):
//   D(r) = argmin_x 1/2 ||x - r||^2 + lam TV(x),  lam = alpha sqrt(tau_r),
// isotropic TV with forward differences and zero difference past the last
// row / column, approximated by K steps of the fast gradient projection on
// the dual (Beck & Teboulle 2009):
//   x(u) = b - lam grad^T u,
//   p_k = P(u_k + grad x(u_k) / (8 lam)),  u_{k+1} = p_k + beta_k (p_k - p_{k-1}),
// p_0 = u_1 = 0, P the pointwise projection onto the unit disc, output
// x(p_K).  The map is those K steps, so its Monte-Carlo divergence is that
// of a fixed deterministic function.
//
// One launch per step over both images (r and r + eps b, blockIdx.z): a
// thread owns one pixel and reads the extrapolated dual u around it (the
// divergence at the pixel and at its lower and right neighbours), forms the
// three values of x it needs, the forward differences, the projected dual
// and the next extrapolation.  u is ping-ponged between steps (neighbours
// read the previous one); p is read and written by its own thread only.
// The step is HBM / latency bound: about 13 floats move per pixel and step.
#include <cmath>

#include "dg_internal.h"

namespace dg {

static constexpr int kTvBX = 64, kTvBY = 4;

struct TvArgs {
  const float* r;    // image 0 input
  float* b1;         // image 1 input r + eps b (written by tv_prep)
  float* p;          // dual p:  [img][comp][N]
  float* ua;         // extrapolated dual, ping
  float* ub;         // pong
  int I;
  int nimg;
  float alpha;
  const double* tau_r;
  const double* eps;
  float* out0;
  float* out1;
};

__device__ __forceinline__ float tv_lambda(const TvArgs& A) {
  const double t = *A.tau_r;
  return t > 0.0 ? A.alpha * (float)sqrt(t) : 0.0f;
}

// b1 = r + eps b; p = u = 0 for both images.
__global__ void __launch_bounds__(256) tv_prep(TvArgs A, uint64_t seed, int iter) {
  const int64_t N = (int64_t)A.I * A.I;
  const float eps = A.nimg > 1 ? (float)(*A.eps) : 0.0f;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (A.nimg > 1) A.b1[k] = __fmaf_rn(eps, probe_sign(seed, iter, (uint64_t)k), A.r[k]);
    for (int m = 0; m < 2 * A.nimg; ++m) {
      A.p[m * N + k] = 0.0f;
      A.ua[m * N + k] = 0.0f;
    }
  }
}

// (grad^T u)(i, j) of one image; u1 / u2 the two components.
__device__ __forceinline__ float tv_adj(const float* __restrict__ u1, const float* __restrict__ u2,
                                        int i, int j, int I) {
  const int64_t k = (int64_t)i * I + j;
  float a = 0.0f;
  if (i > 0) a += u1[k - I];
  if (i < I - 1) a -= u1[k];
  if (j > 0) a += u2[k - 1];
  if (j < I - 1) a -= u2[k];
  return a;
}

__global__ void __launch_bounds__(kTvBX * kTvBY)
tv_step(TvArgs A, const float* __restrict__ usrc, float* __restrict__ udst, float beta) {
  const int I = A.I;
  const int j = blockIdx.x * kTvBX + threadIdx.x;
  const int i = blockIdx.y * kTvBY + threadIdx.y;
  if (i >= I || j >= I) return;
  const float lam = tv_lambda(A);
  if (!(lam > 0.0f)) return;  // identity: tv_final copies the input
  const int img = blockIdx.z;
  const int64_t N = (int64_t)I * I, k = (int64_t)i * I + j;
  const float* b = img ? A.b1 : A.r;
  const float* u1 = usrc + (int64_t)(2 * img) * N;
  const float* u2 = u1 + N;
  const float x0 = b[k] - lam * tv_adj(u1, u2, i, j, I);
  float g1 = 0.0f, g2 = 0.0f;
  if (i < I - 1) g1 = (b[k + I] - lam * tv_adj(u1, u2, i + 1, j, I)) - x0;
  if (j < I - 1) g2 = (b[k + 1] - lam * tv_adj(u1, u2, i, j + 1, I)) - x0;
  const float s = 1.0f / (8.0f * lam);
  const float q1 = u1[k] + g1 * s, q2 = u2[k] + g2 * s;
  const float nrm = fmaxf(1.0f, sqrtf(q1 * q1 + q2 * q2));
  const float n1 = q1 / nrm, n2 = q2 / nrm;
  float* p1 = A.p + (int64_t)(2 * img) * N;
  float* p2 = p1 + N;
  const float o1 = p1[k], o2 = p2[k];
  p1[k] = n1;
  p2[k] = n2;
  float* d1 = udst + (int64_t)(2 * img) * N;
  d1[k] = n1 + beta * (n1 - o1);
  d1[k + N] = n2 + beta * (n2 - o2);
}

// x = b - lam grad^T p (b itself when lam = 0).
__global__ void __launch_bounds__(kTvBX * kTvBY) tv_final(TvArgs A) {
  const int I = A.I;
  const int j = blockIdx.x * kTvBX + threadIdx.x;
  const int i = blockIdx.y * kTvBY + threadIdx.y;
  if (i >= I || j >= I) return;
  const int img = blockIdx.z;
  const int64_t N = (int64_t)I * I, k = (int64_t)i * I + j;
  const float* b = img ? A.b1 : A.r;
  const float lam = tv_lambda(A);
  float x = b[k];
  if (lam > 0.0f) {
    const float* p1 = A.p + (int64_t)(2 * img) * N;
    x -= lam * tv_adj(p1, p1 + N, i, j, I);
  }
  (img ? A.out1 : A.out0)[k] = x;
}

size_t tv_work_bytes(int64_t npix) {
  // b1, then p, ua, ub for two images (2 components each)
  const size_t f = sizeof(float) * (size_t)npix;
  const size_t a = (f + 255) & ~(size_t)255;
  return a + 3 * 4 * a;
}

dg_status tv_check_params(const dg_plan* p, const void* params) {
  DG_ARG_CHECK(params != nullptr, "denoise: TV params must not be NULL");
  const dg_tv_params* tp = (const dg_tv_params*)params;
  DG_ARG_CHECK(tp->alpha >= 0 && std::isfinite(tp->alpha), "denoise: TV alpha must be >= 0");
  DG_ARG_CHECK(tp->iters >= 1 && tp->iters <= 10000, "denoise: TV iters must be in [1, 10000]");
  DG_ARG_CHECK(tp->work != nullptr, "denoise: TV work buffer must not be NULL");
  DG_ARG_CHECK(p->I >= 2, "denoise: TV needs a side of at least 2");
  return DG_OK;
}

dg_status tv_launch_denoise(const dg_plan* p, const void* params, const float* r,
                            const double* tau_r, const double* eps, uint64_t seed, int iter,
                            float* x_den, float* x_pert, hipStream_t st) {
  const dg_tv_params* tp = (const dg_tv_params*)params;
  const int I = p->I;
  const int64_t N = (int64_t)I * I;
  const size_t f = (sizeof(float) * (size_t)N + 255) & ~(size_t)255;
  char* c = (char*)tp->work;
  TvArgs A;
  A.r = r;
  A.b1 = (float*)c;
  A.p = (float*)(c + f);
  A.ua = (float*)(c + f + 4 * f);
  A.ub = (float*)(c + f + 8 * f);
  A.I = I;
  A.nimg = x_pert ? 2 : 1;
  A.alpha = (float)tp->alpha;
  A.tau_r = tau_r;
  A.eps = eps;
  A.out0 = x_den;
  A.out1 = x_pert;
  // regions of f bytes >= N floats; the kernels index component planes N floats apart
  const unsigned int g = (unsigned int)((N + 255) / 256 < 2048 ? (N + 255) / 256 : 2048);
  hipLaunchKernelGGL(tv_prep, dim3(g), dim3(256), 0, st, A, seed, iter);
  DG_LAUNCH_CHECK("tv_prep");
  const dim3 grid((I + kTvBX - 1) / kTvBX, (I + kTvBY - 1) / kTvBY, A.nimg);
  const dim3 block(kTvBX, kTvBY);
  double t = 1.0;
  float* src = A.ua;
  float* dst = A.ub;
  for (int k = 0; k < tp->iters; ++k) {
    const double t1 = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    const float beta = (float)((t - 1.0) / t1);
    t = t1;
    hipLaunchKernelGGL(tv_step, grid, block, 0, st, A, (const float*)src, dst, beta);
    DG_LAUNCH_CHECK("tv_step");
    float* tmp = src;
    src = dst;
    dst = tmp;
  }
  hipLaunchKernelGGL(tv_final, grid, block, 0, st, A);
  DG_LAUNCH_CHECK("tv_final");
  return DG_OK;
}

}  // namespace dg

using namespace dg;

extern "C" size_t dg_tv_workspace_bytes(int64_t n_pixels) {
  return n_pixels > 0 ? tv_work_bytes(n_pixels) : 0;
}
