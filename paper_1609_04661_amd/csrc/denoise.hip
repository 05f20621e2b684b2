// Plug-in denoisers D(r) and the Monte-Carlo divergence (Sec. 4.3, eqs.
// D_in and MC_SURE).  Every denoiser runs its primal input r and the probed
// input r + eps b in one launch (blockIdx.z selects the image); the probe
// b_i = +-1 comes from a counter hash, so it is never stored.
//
//  * Non-local means: 16 x 16 output tile per workgroup, the tile plus the
//    search and patch halos staged in LDS (half-sample symmetric borders).
//    For each search offset the squared differences over the tile plus the
//    patch halo go to LDS, are box-summed separably (rows, then columns), and
//    turned into one weight per output pixel.
//  * Haar soft threshold: the orthonormal 2D Haar pyramid with J levels is
//    local to 2^J x 2^J blocks, so each block is transformed, thresholded and
//    inverted in LDS by one workgroup.
//  * Divergence: div = b^T (D(r + eps b) - D(r)) / (N eps), FP64 sum with a
//    last-block finish that also updates tau_x (Alg. 1 step 4) and applies
//    the damping of x when running inside the iteration.
#include <cmath>

#include "dg_internal.h"

namespace dg {

dg_status launch_zero_u32(unsigned int* p, int n, hipStream_t st);

static constexpr int kTile = 16;
static constexpr int kMaxP = 3, kMaxS = 10;
static constexpr int kRegion = kTile + 2 * (kMaxS + kMaxP);  // 42
static constexpr int kDiff = kTile + 2 * kMaxP;              // 22
static constexpr int kRedBlock = 256;
static constexpr int kRedMaxBlocks = 1024;
static constexpr int kHaarPer = 16;  // (128/2)^2 blocks / 256 threads

// Half-sample symmetric extension (-1 -> 0, I -> I-1), repeated for indices
// more than one image side away, then clamped so every read stays in bounds.
__device__ __forceinline__ int reflect_idx(int k, int I) {
  for (int it = 0; it < 8 && (k < 0 || k >= I); ++it) {
    if (k < 0) k = -k - 1;
    if (k >= I) k = 2 * I - k - 1;
  }
  return min(max(k, 0), I - 1);
}

__global__ void __launch_bounds__(kTile* kTile)
nlm_kernel(const float* __restrict__ r, float* __restrict__ out0, float* __restrict__ out1, int I,
           int P, int S, const double* __restrict__ tau_r_ptr, float hfac,
           const double* __restrict__ eps_ptr, uint64_t seed, int iter) {
  __shared__ float R[kRegion * kRegion];
  __shared__ float D[kDiff * kDiff];
  __shared__ float H[kDiff * kTile];
  const int img = blockIdx.z;
  float* out = img ? out1 : out0;
  const int ty0 = blockIdx.y * kTile, tx0 = blockIdx.x * kTile;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kTile + tx;
  const int H0 = S + P;             // halo
  const int WR = kTile + 2 * H0;    // region width
  const int WD = kTile + 2 * P;     // diff width
  const float eps = img ? (float)(*eps_ptr) : 0.0f;
  for (int e = tid; e < WR * WR; e += kTile * kTile) {
    const int ri = e / WR, rj = e % WR;
    const int gi = reflect_idx(ty0 - H0 + ri, I), gj = reflect_idx(tx0 - H0 + rj, I);
    const int64_t gidx = (int64_t)gi * I + gj;
    float v = r[gidx];
    if (img) v = __fmaf_rn(eps, probe_sign(seed, iter, (uint64_t)gidx), v);
    R[ri * kRegion + rj] = v;
  }
  __syncthreads();
  const double tau_r = *tau_r_ptr;
  const float sig2 = (float)tau_r;
  const float inv_h2 = 1.0f / (hfac * hfac * sig2);
  const float inv_np = 1.0f / (float)((2 * P + 1) * (2 * P + 1));
  const bool active = (ty0 + ty < I) && (tx0 + tx < I);
  float wsum = 0.0f, acc = 0.0f;
  if (!(tau_r > 0.0)) {  // sigma = 0: identity
    if (active) out[(int64_t)(ty0 + ty) * I + tx0 + tx] = R[(H0 + ty) * kRegion + H0 + tx];
    return;
  }
  for (int oi = -S; oi <= S; ++oi) {
    for (int oj = -S; oj <= S; ++oj) {
      for (int e = tid; e < WD * WD; e += kTile * kTile) {
        const int a = e / WD, c = e % WD;
        const float u = R[(S + a) * kRegion + S + c];
        const float v = R[(S + a + oi) * kRegion + S + c + oj];
        const float d = u - v;
        D[a * kDiff + c] = d * d;
      }
      __syncthreads();
      for (int e = tid; e < WD * kTile; e += kTile * kTile) {
        const int a = e / kTile, c = e % kTile;
        float h = 0.0f;
        for (int q = 0; q <= 2 * P; ++q) h += D[a * kDiff + c + q];
        H[a * kTile + c] = h;
      }
      __syncthreads();
      float b = 0.0f;
      for (int q = 0; q <= 2 * P; ++q) b += H[(ty + q) * kTile + tx];
      const float d2 = b * inv_np;
      const float w = __expf(-fmaxf(d2 - 2.0f * sig2, 0.0f) * inv_h2);
      wsum += w;
      acc = __fmaf_rn(w, R[(H0 + ty + oi) * kRegion + H0 + tx + oj], acc);
    }
  }
  if (active) out[(int64_t)(ty0 + ty) * I + tx0 + tx] = acc / wsum;
}

// Haar: one workgroup per B x B block (B = 2^J), dynamic LDS of B*B floats.
__global__ void __launch_bounds__(256)
haar_kernel(const float* __restrict__ r, float* __restrict__ out0, float* __restrict__ out1, int I,
            int J, const double* __restrict__ tau_r_ptr, float alpha,
            const double* __restrict__ eps_ptr, uint64_t seed, int iter) {
  extern __shared__ float T[];
  const int img = blockIdx.z;
  float* out = img ? out1 : out0;
  const int B = 1 << J;
  const int bi = blockIdx.y * B, bj = blockIdx.x * B;
  const float eps = img ? (float)(*eps_ptr) : 0.0f;
  for (int e = threadIdx.x; e < B * B; e += blockDim.x) {
    const int a = e / B, c = e % B;
    const int64_t g = (int64_t)(bi + a) * I + bj + c;
    float v = r[g];
    if (img) v = __fmaf_rn(eps, probe_sign(seed, iter, (uint64_t)g), v);
    T[e] = v;
  }
  __syncthreads();
  // forward: each level works on the top-left n x n block.  A thread reads
  // all of its 2 x 2 blocks into registers before anyone writes, so the
  // in-place scatter to the four quadrants cannot clobber unread inputs.
  for (int n = B; n >= 2; n >>= 1) {
    const int h = n / 2, nblk = h * h;
    float v[kHaarPer][4];
#pragma unroll
    for (int q = 0; q < kHaarPer; ++q) {
      const int e = q * (int)blockDim.x + (int)threadIdx.x;
      if (e < nblk) {
        const int a = e / h, c = e % h;
        const float p00 = T[(2 * a) * B + 2 * c], p01 = T[(2 * a) * B + 2 * c + 1];
        const float p10 = T[(2 * a + 1) * B + 2 * c], p11 = T[(2 * a + 1) * B + 2 * c + 1];
        v[q][0] = 0.5f * (p00 + p01 + p10 + p11);  // LL
        v[q][1] = 0.5f * (p00 - p01 + p10 - p11);  // top-right quadrant
        v[q][2] = 0.5f * (p00 + p01 - p10 - p11);  // bottom-left quadrant
        v[q][3] = 0.5f * (p00 - p01 - p10 + p11);  // HH
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kHaarPer; ++q) {
      const int e = q * (int)blockDim.x + (int)threadIdx.x;
      if (e < nblk) {
        const int a = e / h, c = e % h;
        T[a * B + c] = v[q][0];
        T[a * B + c + h] = v[q][1];
        T[(a + h) * B + c] = v[q][2];
        T[(a + h) * B + c + h] = v[q][3];
      }
    }
    __syncthreads();
  }
  // soft threshold on every coefficient except the single approximation T[0]
  const float lam = alpha * (float)sqrt(*tau_r_ptr);
  for (int e = threadIdx.x; e < B * B; e += blockDim.x) {
    if (e == 0) continue;
    const float w = T[e];
    const float m = fmaxf(fabsf(w) - lam, 0.0f);
    T[e] = copysignf(m, w);
  }
  __syncthreads();
  // inverse
  for (int n = 2; n <= B; n <<= 1) {
    const int h = n / 2, nblk = h * h;
    float v[kHaarPer][4];
#pragma unroll
    for (int q = 0; q < kHaarPer; ++q) {
      const int e = q * (int)blockDim.x + (int)threadIdx.x;
      if (e < nblk) {
        const int a = e / h, c = e % h;
        const float LL = T[a * B + c], TR = T[a * B + c + h];
        const float BL = T[(a + h) * B + c], HH = T[(a + h) * B + c + h];
        v[q][0] = 0.5f * (LL + TR + BL + HH);
        v[q][1] = 0.5f * (LL - TR + BL - HH);
        v[q][2] = 0.5f * (LL + TR - BL - HH);
        v[q][3] = 0.5f * (LL - TR - BL + HH);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kHaarPer; ++q) {
      const int e = q * (int)blockDim.x + (int)threadIdx.x;
      if (e < nblk) {
        const int a = e / h, c = e % h;
        T[(2 * a) * B + 2 * c] = v[q][0];
        T[(2 * a) * B + 2 * c + 1] = v[q][1];
        T[(2 * a + 1) * B + 2 * c] = v[q][2];
        T[(2 * a + 1) * B + 2 * c + 1] = v[q][3];
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < B * B; e += blockDim.x) {
    const int a = e / B, c = e % B;
    out[(int64_t)(bi + a) * I + bj + c] = T[e];
  }
}

// eps = max(eps_rel * max|r|, 1e-12) into *eps_out.
__global__ void __launch_bounds__(kRedBlock)
absmax_kernel(const float* __restrict__ r, int64_t N, double eps_rel, double* eps_out,
              float* __restrict__ partials, unsigned int* counter) {
  __shared__ float red[kRedBlock / 64];
  __shared__ int flag;
  float m = 0.0f;
  for (int64_t k = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; k < N;
       k += (int64_t)gridDim.x * kRedBlock)
    m = fmaxf(m, fabsf(r[k]));
  float bm = block_max(m, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = bm;
  if (last_block(counter, &flag)) {
    float gm = 0.0f;
    for (int k = threadIdx.x; k < (int)gridDim.x; k += blockDim.x) gm = fmaxf(gm, partials[k]);
    gm = block_max(gm, red);
    if (threadIdx.x == 0) {
      double e = eps_rel * (double)gm;
      *eps_out = e > 1e-12 ? e : 1e-12;
      *counter = 0u;
    }
  }
}

// Divergence and (inside the iteration) the tau_x update and damping of x.
//   mode 0: *div_out = div                                  (standalone)
//   mode 1: scal[DIV] = div, scal[TAU_X] updated, x updated (iteration)
__global__ void __launch_bounds__(kRedBlock)
div_kernel(int64_t N, const float* __restrict__ xden, const float* __restrict__ xpert,
           float* __restrict__ x, const double* __restrict__ eps_ptr, double* div_out,
           double* scal, int mode, uint64_t seed, int iter, double eta_x, int t,
           double* __restrict__ partials, unsigned int* counter) {
  __shared__ double red[kRedBlock / 64];
  __shared__ int flag;
  if (mode == 1 && scal[DG_S_STATUS] != 0.0) return;
  const float eta = (float)eta_x;
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; k < N;
       k += (int64_t)gridDim.x * kRedBlock) {
    const float d0 = xden[k];
    const float b = probe_sign(seed, iter, (uint64_t)k);
    acc += (double)(b * (xpert[k] - d0));
    if (mode == 1) x[k] = (t > 0) ? __fmaf_rn(eta, d0, (1.0f - eta) * x[k]) : d0;
  }
  double bs = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = bs;
  if (last_block(counter, &flag)) {
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (unsigned int b = 0; b < gridDim.x; ++b) tot += partials[b];
      const double div = tot / ((double)N * (*eps_ptr));
      if (mode == 0) {
        *div_out = div;
      } else {
        const double tau_r = scal[DG_S_TAU_R];
        double tau_x = div > 0.0 ? tau_r * div : 1e-12 * tau_r;
        if (!(div > 0.0)) scal[DG_S_CLAMPS] += 1.0;
        if (t > 0) tau_x = eta_x * tau_x + (1.0 - eta_x) * scal[DG_S_TAU_X];
        scal[DG_S_DIV] = div;
        scal[DG_S_TAU_X] = tau_x;
        if (!(tau_x > 0.0) || !isfinite(tau_x)) scal[DG_S_STATUS] = (double)(t + 1);
      }
      *counter = 0u;
    }
  }
}

// b_k for Hutchinson's estimator (probe counter k), as floats.
__global__ void probe_kernel(float* __restrict__ b, int64_t N, uint64_t seed, int k) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = probe_sign(seed, k, (uint64_t)i);
}

// ------------------------------------------------------------ launchers

struct DenoiseWork {
  unsigned int* counters;  // 4
  double* dpart;           // kRedMaxBlocks
  float* fpart;            // kRedMaxBlocks
  double* eps;             // 1 (+ spare)
  float* xpert;            // N
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t denoise_work_bytes(const dg_plan* p) {
  return 256 + align256(sizeof(double) * kRedMaxBlocks) + align256(sizeof(float) * kRedMaxBlocks) +
         256 + align256(sizeof(float) * (size_t)p->N);
}

static DenoiseWork carve(const dg_plan* p, void* work) {
  char* c = (char*)work;
  DenoiseWork w;
  w.counters = (unsigned int*)c;
  c += 256;
  w.dpart = (double*)c;
  c += align256(sizeof(double) * kRedMaxBlocks);
  w.fpart = (float*)c;
  c += align256(sizeof(float) * kRedMaxBlocks);
  w.eps = (double*)c;
  c += 256;
  w.xpert = (float*)c;
  return w;
}

unsigned int red_grid(int64_t N) { return grid_for(N, kRedBlock, kRedMaxBlocks); }

dg_status launch_absmax(const float* r, int64_t N, double eps_rel, double* eps_out,
                        float* partials, unsigned int* counter, hipStream_t st) {
  hipLaunchKernelGGL(absmax_kernel, dim3(red_grid(N)), dim3(kRedBlock), 0, st, r, N, eps_rel,
                     eps_out, partials, counter);
  DG_LAUNCH_CHECK("absmax_kernel");
  return DG_OK;
}

static int haar_levels(const dg_plan* p, const dg_haar_params* hp) {
  int J = hp->levels;
  if (J <= 0) {
    J = 0;
    while ((1 << (J + 1)) <= p->I) ++J;  // log2 I
    J = J - 2;
    if (J < 1) J = 1;
  }
  return J;
}

dg_status check_denoise_params(const dg_plan* p, int kind, const void* params) {
  DG_ARG_CHECK(params != nullptr, "denoise: params must not be NULL");
  if (kind == DG_DEN_NLM) {
    const dg_nlm_params* np = (const dg_nlm_params*)params;
    DG_ARG_CHECK(np->patch_radius >= 0 && np->patch_radius <= kMaxP,
                 "denoise: NLM patch radius must be in [0, 3]");
    DG_ARG_CHECK(np->search_radius >= 0 && np->search_radius <= kMaxS,
                 "denoise: NLM search radius must be in [0, 10]");
    DG_ARG_CHECK(np->search_radius + np->patch_radius < p->I, "denoise: NLM window exceeds image");
    DG_ARG_CHECK(np->hfac > 0 && std::isfinite(np->hfac), "denoise: NLM hfac must be > 0");
  } else if (kind == DG_DEN_HAAR) {
    const dg_haar_params* hp = (const dg_haar_params*)params;
    DG_ARG_CHECK(hp->alpha >= 0 && std::isfinite(hp->alpha), "denoise: Haar alpha must be >= 0");
    int J = haar_levels(p, hp);
    if ((p->I & (p->I - 1)) != 0 || J > 7 || (1 << J) > p->I) {
      set_error("denoise: Haar needs a power-of-two side and 2^levels <= min(I, 128)");
      return DG_ERR_UNSUPPORTED;
    }
  } else if (kind == DG_DEN_CNN) {
    set_error("denoise: CNN kind is dispatched by the CNN module");
    return DG_ERR_UNSUPPORTED;
  } else {
    set_error("denoise: unknown kind");
    return DG_ERR_ARG;
  }
  return DG_OK;
}

// Runs D on r (into x_den) and, when probed, on r + eps b (into x_pert).
dg_status launch_denoiser(const dg_plan* p, int kind, const void* params, const float* r,
                          const double* tau_r, const double* eps, uint64_t seed, int iter,
                          float* x_den, float* x_pert, hipStream_t st) {
  const int nimg = x_pert ? 2 : 1;
  if (kind == DG_DEN_NLM) {
    const dg_nlm_params* np = (const dg_nlm_params*)params;
    dim3 grid((p->I + kTile - 1) / kTile, (p->I + kTile - 1) / kTile, nimg);
    hipLaunchKernelGGL(nlm_kernel, grid, dim3(kTile, kTile), 0, st, r, x_den, x_pert, p->I,
                       np->patch_radius, np->search_radius, tau_r, (float)np->hfac, eps, seed,
                       iter);
    DG_LAUNCH_CHECK("nlm_kernel");
    return DG_OK;
  }
  if (kind == DG_DEN_HAAR) {
    const dg_haar_params* hp = (const dg_haar_params*)params;
    const int J = haar_levels(p, hp);
    const int B = 1 << J;
    dim3 grid(p->I / B, p->I / B, nimg);
    hipLaunchKernelGGL(haar_kernel, grid, dim3(256), sizeof(float) * B * B, st, r, x_den, x_pert,
                       p->I, J, tau_r, (float)hp->alpha, eps, seed, iter);
    DG_LAUNCH_CHECK("haar_kernel");
    return DG_OK;
  }
  set_error("denoise: unsupported kind");
  return DG_ERR_UNSUPPORTED;
}

dg_status launch_div(const dg_plan* p, const float* xden, const float* xpert, float* x,
                     const double* eps, double* div_out, double* scal, int mode, uint64_t seed,
                     int iter, double eta_x, int t, double* partials, unsigned int* counter,
                     hipStream_t st) {
  hipLaunchKernelGGL(div_kernel, dim3(red_grid(p->N)), dim3(kRedBlock), 0, st, p->N, xden, xpert,
                     x, eps, div_out, scal, mode, seed, iter, eta_x, t, partials, counter);
  DG_LAUNCH_CHECK("div_kernel");
  return DG_OK;
}

dg_status launch_probe(float* b, int64_t N, uint64_t seed, int k, hipStream_t st) {
  hipLaunchKernelGGL(probe_kernel, dim3(red_grid(N)), dim3(256), 0, st, b, N, seed, k);
  DG_LAUNCH_CHECK("probe_kernel");
  return DG_OK;
}

// CNN module hooks (defined in cnn.hip).
dg_status cnn_check_params(const dg_plan* p, const void* params);
dg_status cnn_launch_denoise(const dg_plan* p, const void* params, const float* r,
                             const double* eps, uint64_t seed, int iter, float* x_den,
                             float* x_pert, double* div_dot_out, hipStream_t st);

}  // namespace dg

using namespace dg;

extern "C" dg_status denoise(const dg_plan* p, int32_t kind, const void* params, const float* r,
                             const double* tau_r, uint64_t probe_seed, int32_t iter,
                             double eps_rel, float* x_out, double* div_out, void* work,
                             void* stream) {
  DG_ARG_CHECK(p && r && tau_r && x_out && work, "denoise: null argument");
  DG_ARG_CHECK((const void*)r != (const void*)x_out, "denoise: r and x_out alias");
  DG_ARG_CHECK(eps_rel > 0 && std::isfinite(eps_rel), "denoise: eps_rel must be > 0");
  hipStream_t st = (hipStream_t)stream;
  dg_status rc;
  if (kind == DG_DEN_CNN) {
    rc = cnn_check_params(p, params);
  } else {
    rc = check_denoise_params(p, kind, params);
  }
  if (rc != DG_OK) return rc;
  DenoiseWork w = carve(p, work);
  if ((rc = launch_zero_u32(w.counters, 4, st)) != DG_OK) return rc;
  float* xpert = nullptr;
  if (div_out) {
    if ((rc = launch_absmax(r, p->N, eps_rel, w.eps, w.fpart, w.counters + 0, st)) != DG_OK)
      return rc;
    xpert = w.xpert;
  }
  if (kind == DG_DEN_CNN) {
    rc = cnn_launch_denoise(p, params, r, w.eps, probe_seed, iter, x_out, xpert, nullptr, st);
  } else {
    rc = launch_denoiser(p, kind, params, r, tau_r, w.eps, probe_seed, iter, x_out, xpert, st);
  }
  if (rc != DG_OK) return rc;
  if (div_out)
    return launch_div(p, x_out, xpert, nullptr, w.eps, div_out, nullptr, 0, probe_seed, iter, 1.0,
                      0, w.dpart, w.counters + 1, st);
  return DG_OK;
}
