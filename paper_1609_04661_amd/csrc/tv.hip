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
// Up to kTvSteps dual steps per launch (both images, blockIdx.z): a
// 768-thread workgroup owns a 32 x 32 output tile and loads the dual state (p, u) and
// the input of the tile plus a halo of kTvSteps pixels into LDS / registers.
// One step's new u at a pixel depends on u within Chebyshev distance 1, so
// after s steps in the launch every pixel at least s from the region's edge
// is exact and the tile itself is exact after kTvSteps; only the tile's
// state goes back to memory (ping-pong buffers: neighbouring workgroups
// read their halos from the previous launch's state).  A step is two
// phases with a workgroup barrier each: x = b - lam grad^T u for every
// region pixel into LDS, then the forward differences of x, the projected
// dual and its extrapolation.  The arithmetic per pixel and step is that of
// one plain step, so the result does not depend on how steps are grouped.
#include <cmath>
#include <utility>

#include "dg_internal.h"

namespace dg {

static constexpr int kTvBX = 64, kTvBY = 4;

struct TvArgs {
  const float* r;    // image 0 input
  float* b1;         // image 1 input r + eps b (written by tv_prep)
  float* pa;         // dual p, ping: [img][comp][N]
  float* pb;         // pong
  float* ua;         // extrapolated dual u, ping
  float* ub;         // pong
  const float* pfin; // the dual after the last step (tv_final)
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

// b1 = r + eps b; p = u = 0 for both images (buffers pa, ua).
__global__ void __launch_bounds__(256) tv_prep(TvArgs A, uint64_t seed, int iter) {
  const int64_t N = (int64_t)A.I * A.I;
  const float eps = A.nimg > 1 ? (float)(*A.eps) : 0.0f;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (A.nimg > 1) A.b1[k] = __fmaf_rn(eps, probe_sign(seed, iter, (uint64_t)k), A.r[k]);
    for (int m = 0; m < 2 * A.nimg; ++m) {
      A.pa[m * N + k] = 0.0f;
      A.ua[m * N + k] = 0.0f;
    }
  }
}

// (grad^T p)(i, j) of one image from global memory; p1 / p2 the components.
__device__ __forceinline__ float tv_adj(const float* __restrict__ p1, const float* __restrict__ p2,
                                        int i, int j, int I) {
  const int64_t k = (int64_t)i * I + j;
  float a = 0.0f;
  if (i > 0) a += p1[k - I];
  if (i < I - 1) a -= p1[k];
  if (j > 0) a += p2[k - 1];
  if (j < I - 1) a -= p2[k];
  return a;
}

static constexpr int kTvTile = 32, kTvSteps = 8;
static constexpr int kTvRegion = kTvTile + 2 * kTvSteps;         // 48
static constexpr int kTvPix = kTvRegion * kTvRegion;              // 2304
static constexpr int kTvThreads = 768;                            // 12 wavefronts
static constexpr int kTvPer = kTvPix / kTvThreads;                // 3
static_assert(kTvPix % kTvThreads == 0, "region pixels split evenly over the threads");

struct TvBetas {
  float b[kTvSteps];
};

// nsteps (1 .. kTvSteps) dual steps on one 32 x 32 tile of one image:
// state in from (psrc, usrc), the tile's state out to (pdst, udst).
__global__ void __launch_bounds__(kTvThreads)
tv_steps(TvArgs A, const float* __restrict__ psrc, const float* __restrict__ usrc,
         float* __restrict__ pdst, float* __restrict__ udst, int nsteps, TvBetas betas) {
  __shared__ float sU1[kTvPix], sU2[kTvPix], sX[kTvPix], sB[kTvPix];
  const float lam = tv_lambda(A);
  if (!(lam > 0.0f)) return;  // identity: tv_final copies the input
  const int I = A.I, img = blockIdx.z;
  const int64_t N = (int64_t)I * I;
  const int gi0 = blockIdx.y * kTvTile - kTvSteps, gj0 = blockIdx.x * kTvTile - kTvSteps;
  const float* b = img ? A.b1 : A.r;
  const float* pin1 = psrc + (int64_t)(2 * img) * N;
  const float* uin1 = usrc + (int64_t)(2 * img) * N;
  float p1[kTvPer], p2[kTvPer];
  // per owned pixel, which neighbours its step reads: bit 0 up, 1 here
  // (first component), 2 left, 3 here (second), 4 down, 5 right
  unsigned nb[kTvPer];
  // load the region (zeros outside the image)
#pragma unroll
  for (int q = 0; q < kTvPer; ++q) {
    const int e = q * kTvThreads + threadIdx.x;
    const int ri = e / kTvRegion, rj = e - ri * kTvRegion;
    const int gi = gi0 + ri, gj = gj0 + rj;
    nb[q] = (gi > 0 && ri > 0 ? 1u : 0u) | (gi < I - 1 ? 2u : 0u) | (gj > 0 && rj > 0 ? 4u : 0u) |
            (gj < I - 1 ? 8u : 0u) | (gi < I - 1 && ri < kTvRegion - 1 ? 16u : 0u) |
            (gj < I - 1 && rj < kTvRegion - 1 ? 32u : 0u);
    float vb = 0.0f, vu1 = 0.0f, vu2 = 0.0f, vp1 = 0.0f, vp2 = 0.0f;
    if ((unsigned)gi < (unsigned)I && (unsigned)gj < (unsigned)I) {
      const int64_t k = (int64_t)gi * I + gj;
      vb = b[k];
      vu1 = uin1[k];
      vu2 = uin1[k + N];
      vp1 = pin1[k];
      vp2 = pin1[k + N];
    }
    sB[e] = vb;
    sU1[e] = vu1;
    sU2[e] = vu2;
    p1[q] = vp1;
    p2[q] = vp2;
  }
  __syncthreads();
  const float s8 = 1.0f / (8.0f * lam);
  for (int st = 0; st < nsteps; ++st) {
    // x = b - lam grad^T u over the region (neighbour reads clamped to it)
#pragma unroll
    for (int q = 0; q < kTvPer; ++q) {
      const int e = q * kTvThreads + threadIdx.x;
      float a = 0.0f;
      if (nb[q] & 1u) a += sU1[e - kTvRegion];
      if (nb[q] & 2u) a -= sU1[e];
      if (nb[q] & 4u) a += sU2[e - 1];
      if (nb[q] & 8u) a -= sU2[e];
      sX[e] = sB[e] - lam * a;
    }
    __syncthreads();
    const float beta = betas.b[st];
#pragma unroll
    for (int q = 0; q < kTvPer; ++q) {
      const int e = q * kTvThreads + threadIdx.x;
      const float x0 = sX[e];
      float g1 = 0.0f, g2 = 0.0f;
      if (nb[q] & 16u) g1 = sX[e + kTvRegion] - x0;
      if (nb[q] & 32u) g2 = sX[e + 1] - x0;
      const float q1 = sU1[e] + g1 * s8, q2 = sU2[e] + g2 * s8;
      const float nrm = fmaxf(1.0f, sqrtf(q1 * q1 + q2 * q2));
      const float n1 = q1 / nrm, n2 = q2 / nrm;
      sU1[e] = n1 + beta * (n1 - p1[q]);
      sU2[e] = n2 + beta * (n2 - p2[q]);
      p1[q] = n1;
      p2[q] = n2;
    }
    __syncthreads();
  }
  // the tile's state back to memory
  float* pout1 = pdst + (int64_t)(2 * img) * N;
  float* uout1 = udst + (int64_t)(2 * img) * N;
#pragma unroll
  for (int q = 0; q < kTvPer; ++q) {
    const int e = q * kTvThreads + threadIdx.x;
    const int ri = e / kTvRegion, rj = e - ri * kTvRegion;
    const int gi = gi0 + ri, gj = gj0 + rj;
    const bool inner = ri >= kTvSteps && ri < kTvSteps + kTvTile && rj >= kTvSteps &&
                       rj < kTvSteps + kTvTile;
    if (inner && gi < I && gj < I) {
      const int64_t k = (int64_t)gi * I + gj;
      pout1[k] = p1[q];
      pout1[k + N] = p2[q];
      uout1[k] = sU1[e];
      uout1[k + N] = sU2[e];
    }
  }
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
    const float* p1 = A.pfin + (int64_t)(2 * img) * N;
    x -= lam * tv_adj(p1, p1 + N, i, j, I);
  }
  (img ? A.out1 : A.out0)[k] = x;
}

size_t tv_work_bytes(int64_t npix) {
  // b1, then pa, pb, ua, ub for two images (2 components each)
  const size_t f = sizeof(float) * (size_t)npix;
  const size_t a = (f + 255) & ~(size_t)255;
  return a + 4 * 4 * a;
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
  A.pa = (float*)(c + f);
  A.pb = (float*)(c + 5 * f);
  A.ua = (float*)(c + 9 * f);
  A.ub = (float*)(c + 13 * f);
  A.pfin = A.pa;
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
  const dim3 tgrid((I + kTvTile - 1) / kTvTile, (I + kTvTile - 1) / kTvTile, A.nimg);
  double t = 1.0;
  float *psrc = A.pa, *pdst = A.pb, *usrc = A.ua, *udst = A.ub;
  for (int k0 = 0; k0 < tp->iters; k0 += kTvSteps) {
    const int ns = tp->iters - k0 < kTvSteps ? tp->iters - k0 : kTvSteps;
    TvBetas be{};
    for (int m = 0; m < ns; ++m) {
      const double t1 = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
      be.b[m] = (float)((t - 1.0) / t1);
      t = t1;
    }
    hipLaunchKernelGGL(tv_steps, tgrid, dim3(kTvThreads), 0, st, A, (const float*)psrc,
                       (const float*)usrc, pdst, udst, ns, be);
    DG_LAUNCH_CHECK("tv_steps");
    std::swap(psrc, pdst);
    std::swap(usrc, udst);
  }
  A.pfin = psrc;
  const dim3 grid((I + kTvBX - 1) / kTvBX, (I + kTvBY - 1) / kTvBY, A.nimg);
  hipLaunchKernelGGL(tv_final, grid, dim3(kTvBX, kTvBY), 0, st, A);
  DG_LAUNCH_CHECK("tv_final");
  return DG_OK;
}

}  // namespace dg

using namespace dg;

extern "C" size_t dg_tv_workspace_bytes(int64_t n_pixels) {
  return n_pixels > 0 ? tv_work_bytes(n_pixels) : 0;
}
