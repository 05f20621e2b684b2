// Plug-in denoisers D(r) and the Monte-Carlo divergence (Sec. 4.3, eqs.
// D_in and MC_SURE).  Every denoiser runs its primal input r and the probed
// input r + eps b in one launch (blockIdx.z selects the image); the probe
// b_i = +-1 comes from a counter hash, so it is never stored.
//
//  * Non-local means: 32 x 32 output tile per workgroup staged in LDS with
//    its halos (half-sample symmetric borders); register-blocked patch
//    distances with sliding box sums (see nlm_kernel).
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

// proximal TV (tv.hip)
dg_status tv_check_params(const dg_plan* p, const void* params);
dg_status tv_launch_denoise(const dg_plan* p, const void* params, const float* r,
                            const double* tau_r, const double* eps, uint64_t seed, int iter,
                            float* x_den, float* x_pert, hipStream_t st);
// proximal TV in the (V^T V)^-1 metric (tvw.hip)
dg_status tvw_check_params(const dg_plan* p, const void* params);
dg_status bm3d_check_params(const dg_plan* p, const void* params);
dg_status bm3d_launch_denoise(const dg_plan* p, const void* params, const float* r,
                              const double* tau_r, const double* eps, uint64_t seed, int iter,
                              float* x_den, float* x_pert, hipStream_t st);
dg_status tvw_launch_denoise(const dg_plan* p, const void* params, const float* r,
                             const double* tau_r, const double* eps, uint64_t seed, int iter,
                             float* x_den, float* x_pert, hipStream_t st);

static constexpr int kMaxP = 3, kMaxS = 10;
static constexpr int kNlmTile = 32;
static constexpr int kNlmRegion = kNlmTile + 2 * (kMaxS + kMaxP);  // 58
static_assert(kNlmRegion <= 64, "the staging loop gives each region column a lane");
static constexpr int kNlmPitch = kNlmRegion + 1;
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

// Non-local means, register-blocked.  A workgroup owns a 32 x 32 output
// tile and stages the tile plus its search and patch halos in LDS.  Its
// W wavefronts split the offsets of the search window evenly, taken in
// row-major order (a wavefront's share may start and end inside a row: the
// 441 offsets of S = 10 give 55 or 56 per wavefront with W = 8, where whole
// rows gave 3 rows = 63 to each of 7 wavefronts and left an eighth of the
// wave slots idle); each thread
// owns a 2-wide, 8-tall block of outputs and keeps the (8 + 2P) x (2 + 2P)
// input pixels its patches cover in registers (own).  Along a row of the
// search window (oj = -S .. S) the shifted region slides right by one
// column per offset, so it lives in a ring of registers and only its new
// column is read from LDS (8 + 2P values per offset instead of
// (8 + 2P) (2 + 2P)); the ring slot of a column is static because the oj
// loop is unrolled by the ring width.  Per offset the thread forms the
// differences, sums their squares along each row (the two outputs of a row
// share the middle 2P squares, accumulated with fused multiply-adds), sums
// those vertically with a sliding sum, and turns each sum into a weight.  The wavefronts' partial
// sums are added in a fixed order at the end.
// The number of wavefronts W that split a tile's offsets is a tuning
// variant (0: W = 8, 1: W = 4): a workgroup of 4 holds half the LDS for
// its partial sums, so two fit a compute unit where one of 8 does (the
// register budget allows 8 wavefronts either way); the larger workgroup
// fills more compute units when an image has few tiles.
static constexpr int kNlmBX = 2, kNlmBY = 8;
static_assert(kNlmBX == 2, "the row sums below are written for two outputs per row");
__host__ __device__ constexpr int nlm_waves(int variant) { return variant == 1 ? 4 : 8; }
// The search loop and the per-output normalisation of nlm_body.
// R holds the region scaled by sqrt(c1) (nlm_consts), so a patch's sum of
// squared differences is c1 S directly; the sliding sums start at -c2, and
// the weight 2^-max(c1 S - c2, 0) is one exp with a negated input and its
// output clamped to [0, 1].  The weighted mean is unscaled by inv_k.
template <int P, int W, class Emit>
__device__ __forceinline__ void nlm_search(const NlmArgs& Ar, const float* R,
                                           float (*red)[64][2 * kNlmBX * kNlmBY], int ox0, int oy0,
                                           int g, int lane, float c2, float inv_k, int ty0,
                                           int tx0, Emit& emit) {
  constexpr int BX = kNlmBX, BY = kNlmBY;
  constexpr int WX = BX + 2 * P, WY = BY + 2 * P;
  const int I = Ar.I, S = Ar.S;
  float own[WY][WX];
#pragma unroll
  for (int a = 0; a < WY; ++a)
#pragma unroll
    for (int c = 0; c < WX; ++c) own[a][c] = R[(S + oy0 + a) * kNlmPitch + S + ox0 + c];
  float wsum[BY][BX], acc[BY][BX];
#pragma unroll
  for (int a = 0; a < BY; ++a)
#pragma unroll
    for (int c = 0; c < BX; ++c) wsum[a][c] = acc[a][c] = 0.0f;
  const int nside = 2 * S + 1, n2 = nside * nside;
  // this wavefront's offsets e = (oi + S) nside + (oj + S), e0 <= e < e1
  const int e0 = g * n2 / W, e1 = (g + 1) * n2 / W;
  for (int row = e0 / nside; row * nside < e1; ++row) {
    const int oi = row - S;
    const int ja = max(e0 - row * nside, 0), jb = min(e1 - row * nside, nside) - 1;
    if (ja > jb) continue;  // wavefront-uniform
    // shifted region of step t = oj + S: column c of it is LDS column
    // ox0 + t + c of row S + oy0 + a + oi, held in ring slot (t + c) % WX;
    // before step ja the slots hold columns ja .. ja + WX - 2
    const float* rowbase = R + (S + oy0 + oi) * kNlmPitch + ox0;
    float win[WY][WX];
    const int jr = ja % WX;
#pragma unroll
    for (int sl = 0; sl < WX; ++sl) {
      const int pc = ja + (sl - jr + WX) % WX;  // the column of ring slot sl
      if (pc < ja + WX - 1) {
#pragma unroll
        for (int a = 0; a < WY; ++a) win[a][sl] = rowbase[a * kNlmPitch + pc];
      }
    }
    for (int t0 = ja - jr; t0 <= jb; t0 += WX) {
#pragma unroll
      for (int tau = 0; tau < WX; ++tau) {
        const int t = t0 + tau;
        if (t >= ja && t <= jb) {  // wavefront-uniform
#pragma unroll
          for (int a = 0; a < WY; ++a)
            win[a][(tau + WX - 1) % WX] = rowbase[a * kNlmPitch + t + WX - 1];
          float h[WY][BX];
#pragma unroll
          for (int a = 0; a < WY; ++a) {
            float d[WX];
#pragma unroll
            for (int c = 0; c < WX; ++c) d[c] = own[a][c] - win[a][(tau + c) % WX];
            // the two outputs' row sums share the squares of d[1 .. 2P]:
            // one multiply and 2P + 1 fused multiply-adds for both
            float mid = d[1] * d[1];
#pragma unroll
            for (int q = 2; q <= 2 * P; ++q) mid = __fmaf_rn(d[q], d[q], mid);
            h[a][0] = __fmaf_rn(d[0], d[0], mid);
            h[a][1] = __fmaf_rn(d[2 * P + 1], d[2 * P + 1], mid);
          }
#pragma unroll
          for (int c = 0; c < BX; ++c) {
            float v = -c2;
#pragma unroll
            for (int q = 0; q <= 2 * P; ++q) v += h[q][c];
#pragma unroll
            for (int a = 0; a < BY; ++a) {
              if (a > 0) v += h[a + 2 * P][c] - h[a - 1][c];
              // v = c1 S - c2; 2^-max(v, 0) = min(2^-v, 1): the negation and
              // the clamp to [0, 1] fold into the exp instruction's modifiers
              const float w = fminf(fmaxf(__builtin_amdgcn_exp2f(-v), 0.0f), 1.0f);
              wsum[a][c] += w;
              acc[a][c] = __fmaf_rn(w, win[a + P][(tau + c + P) % WX], acc[a][c]);
            }
          }
        }
      }
    }
  }
  // add the wavefronts' partial sums in a fixed order
#pragma unroll
  for (int a = 0; a < BY; ++a)
#pragma unroll
    for (int c = 0; c < BX; ++c) {
      red[g][lane][2 * (a * BX + c)] = wsum[a][c];
      red[g][lane][2 * (a * BX + c) + 1] = acc[a][c];
    }
  __syncthreads();
  // thread (g, lane) finalises outputs k = g, g + W, ... of block `lane`
  for (int k = g; k < BX * BY; k += W) {
    float ws = 0.0f, ac = 0.0f;
#pragma unroll
    for (int gg = 0; gg < W; ++gg) {
      ws += red[gg][lane][2 * k];
      ac += red[gg][lane][2 * k + 1];
    }
    const int a = k / BX, c = k % BX;
    const int gy = ty0 + oy0 + a, gx = tx0 + ox0 + c;
    if (gy < I && gx < I) emit(gy, gx, (ac / ws) * inv_k);
  }
}

template <int P, int W>
__device__ void nlm_body(const NlmArgs& Ar, int bx, int by, int img, uint64_t seed, int iter,
                         double eta_x, int t, float* R, float (*red)[64][2 * kNlmBX * kNlmBY]) {
  __shared__ double dsh[W + 1];
  constexpr int BX = kNlmBX, BY = kNlmBY;
  const float* __restrict__ r = Ar.r;
  const int I = Ar.I, S = Ar.S;
  const double* __restrict__ tau_r_ptr = Ar.tau_r;
  float* out = img ? Ar.out1 : Ar.out0;
  const int ty0 = by * kNlmTile, tx0 = bx * kNlmTile;
  const int H0 = S + P;
  const int WR = kNlmTile + 2 * H0;
  // fused divergence: off once the status word is set (the recursion is
  // frozen, as in the separate divergence pass)
  const bool fuse = Ar.x != nullptr && Ar.scal[DG_S_STATUS] == 0.0;
  float eps = 0.0f;
  double eps_d = 0.0;
  if (Ar.eps_part) {
    // Monte-Carlo step from the preconditioner's per-workgroup max |r|
    // (finished here rather than in a launch of its own); red is free yet
    float* sh = &red[0][0][0];
    const float gm = finish_max(Ar.eps_part, Ar.eps_n, sh);
    if (threadIdx.x == 0) {
      double e = Ar.eps_rel * (double)gm;
      e = e > 1e-12 ? e : 1e-12;
      if (bx == 0 && by == 0 && img == 0) *Ar.eps_out = e;
      dsh[0] = e;
    }
    __syncthreads();
    eps_d = dsh[0];
    eps = img ? (float)eps_d : 0.0f;
    __syncthreads();
  } else if (img || fuse) {
    eps_d = *Ar.eps;
    if (img) eps = (float)eps_d;
  }
  // w = exp(-max(S / n_p - 2 sigma^2, 0) / h^2) = 2^-max(c1 S - c2, 0) with
  // c1 = log2(e) / (n_p h^2) and c2 = log2(e) 2 sigma^2 / h^2 (S the patch
  // sum of squared differences over n_p pixels, h = hfac sigma, sigma^2 =
  // tau_r).  The region is stored scaled by k = sqrt(c1).  sigma = 0 (or a
  // sigma^2 below FP32's range) is the identity.
  const double tau_r = *tau_r_ptr;
  const float sig2 = (float)tau_r;
  const float l2e_h2 = 1.4426950408889634f / (Ar.hfac * Ar.hfac * sig2);
  const float c1 = l2e_h2 / (float)((2 * P + 1) * (2 * P + 1));
  const bool smooth = sig2 > 0.0f && c1 <= 3.0e38f;
  const float kscale = smooth ? sqrtf(c1) : 1.0f;
  const float c2 = l2e_h2 * 2.0f * sig2;
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  // the region, a row per wavefront and a column per lane (WR <= 58 < 64):
  // each lane reflects its column once, each wavefront its row once per row
  if (lane < WR) {
    const int gj = reflect_idx(tx0 - H0 + lane, I);
    for (int ri = g; ri < WR; ri += W) {
      const int gi = reflect_idx(ty0 - H0 + ri, I);
      const int64_t gidx = (int64_t)gi * I + gj;
      float v = r[gidx];
      if (img) v = __fmaf_rn(eps, probe_sign(seed, iter, (uint64_t)gidx), v);
      R[ri * kNlmPitch + lane] = v * kscale;
    }
  }
  __syncthreads();
  const int ox0 = (lane & 15) * BX, oy0 = (lane >> 4) * BY;  // tile-relative block origin
  // an output value: stored, and with the fused divergence, x damped towards
  // D(r) (image 0) and -+ b v added to this thread's partial
  const float eta = (float)eta_x;
  double dacc = 0.0;
  auto emit = [&](int gy, int gx, float v) {
    const int64_t gidx = (int64_t)gy * I + gx;
    out[gidx] = v;
    if (fuse) {
      const float b = probe_sign(seed, iter, (uint64_t)gidx);
      if (img) {
        dacc += (double)(b * v);
      } else {
        dacc -= (double)(b * v);
        Ar.x[gidx] = (t > 0) ? __fmaf_rn(eta, v, (1.0f - eta) * Ar.x[gidx]) : v;
      }
    }
  };
  if (!smooth) {  // sigma = 0: identity (the region is unscaled)
    if (g == 0)
      for (int a = 0; a < BY; ++a)
        for (int c = 0; c < BX; ++c) {
          const int gy = ty0 + oy0 + a, gx = tx0 + ox0 + c;
          if (gy < I && gx < I) emit(gy, gx, R[(H0 + oy0 + a) * kNlmPitch + H0 + ox0 + c]);
        }
  } else {
    nlm_search<P, W>(Ar, R, red, ox0, oy0, g, lane, c2, 1.0f / kscale, ty0, tx0, emit);
  }
  if (!fuse) return;
  // the workgroup's partial of b^T (D(r + eps b) - D(r)); the next launch
  // sums them (DivFinish)
  const double bs = block_sum(dacc, dsh);
  const int g2 = (I + kNlmTile - 1) / kNlmTile;
  if (threadIdx.x == 0) Ar.div_part[(img * g2 + by) * g2 + bx] = bs;
}

template <int P, int W>
__global__ void __launch_bounds__(64 * W)
nlm_kernel(NlmArgs A, uint64_t seed, int iter, double eta_x, int t) {
  __shared__ float R[kNlmRegion * kNlmPitch];
  __shared__ float red[W][64][2 * kNlmBX * kNlmBY];
  nlm_body<P, W>(A, blockIdx.x, blockIdx.y, blockIdx.z, seed, iter, eta_x, t, R, red);
}
template <int P, int W>
__global__ void __launch_bounds__(64 * W)
nlm_batch(const NlmArgs* __restrict__ T, const int* __restrict__ prefix, int n, uint64_t seed,
          int iter, double eta_x, int t) {
  __shared__ float R[kNlmRegion * kNlmPitch];
  __shared__ float red[W][64][2 * kNlmBX * kNlmBY];
  const int s = slice_of(prefix, n, blockIdx.x);
  const NlmArgs A = T[s];
  const int local = blockIdx.x - prefix[s];
  const int g = (A.I + kNlmTile - 1) / kNlmTile;
  nlm_body<P, W>(A, local % g, (local / g) % g, local / (g * g), seed, iter, eta_x, t, R, red);
}

// Launch of the single-slice / batched NLM kernel for patch radius P (1, 2,
// else 3) and tuning variant v.
template <int W>
static void nlm_launch_w(int P, dim3 grid, hipStream_t st, const NlmArgs& A, uint64_t seed,
                         int iter, double eta_x, int t) {
  if (P == 1)
    hipLaunchKernelGGL((nlm_kernel<1, W>), grid, dim3(64 * W), 0, st, A, seed, iter, eta_x, t);
  else if (P == 2)
    hipLaunchKernelGGL((nlm_kernel<2, W>), grid, dim3(64 * W), 0, st, A, seed, iter, eta_x, t);
  else
    hipLaunchKernelGGL((nlm_kernel<3, W>), grid, dim3(64 * W), 0, st, A, seed, iter, eta_x, t);
}
static void nlm_launch(int v, int P, dim3 grid, hipStream_t st, const NlmArgs& A, uint64_t seed,
                       int iter, double eta_x, int t) {
  if (nlm_waves(v) == 4)
    nlm_launch_w<4>(P, grid, st, A, seed, iter, eta_x, t);
  else
    nlm_launch_w<8>(P, grid, st, A, seed, iter, eta_x, t);
}
template <int W>
static void nlm_batch_launch_w(int P, int total, hipStream_t st, const NlmArgs* T,
                               const int* prefix, int n, uint64_t seed, int iter, double eta_x,
                               int t) {
  if (P == 1)
    hipLaunchKernelGGL((nlm_batch<1, W>), dim3(total), dim3(64 * W), 0, st, T, prefix, n, seed,
                       iter, eta_x, t);
  else if (P == 2)
    hipLaunchKernelGGL((nlm_batch<2, W>), dim3(total), dim3(64 * W), 0, st, T, prefix, n, seed,
                       iter, eta_x, t);
  else
    hipLaunchKernelGGL((nlm_batch<3, W>), dim3(total), dim3(64 * W), 0, st, T, prefix, n, seed,
                       iter, eta_x, t);
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
absmax_kernel(const float* __restrict__ r, int64_t N, float* __restrict__ partials) {
  __shared__ float red[kRedBlock / 64];
  float m = 0.0f;
  for (int64_t k = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; k < N;
       k += (int64_t)gridDim.x * kRedBlock)
    m = fmaxf(m, fabsf(r[k]));
  float bm = block_max(m, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = bm;
}

// Divergence and (inside the iteration) the tau_x update and damping of x.
//   mode 0: *div_out = div                                  (standalone)
//   mode 1: scal[DIV] = div, scal[TAU_X] updated, x updated (iteration)
__device__ void div_body(const DivArgs& A, int blk, int mode, uint64_t seed, int iter,
                         double eta_x, int t, double* red) {
  if (mode == 1 && A.scal[DG_S_STATUS] != 0.0) return;
  const float eta = (float)eta_x;
  double acc = 0.0;
  for (int64_t k = (int64_t)blk * kRedBlock + threadIdx.x; k < A.N;
       k += (int64_t)A.nblk * kRedBlock) {
    const float d0 = A.xden[k];
    const float b = probe_sign(seed, iter, (uint64_t)k);
    acc += (double)(b * (A.xpert[k] - d0));
    if (mode == 1) A.x[k] = (t > 0) ? __fmaf_rn(eta, d0, (1.0f - eta) * A.x[k]) : d0;
  }
  double bs = block_sum(acc, red);
  if (threadIdx.x == 0) A.partials[blk] = bs;
}

__device__ void div_finish_body(const DivArgs& A, int mode, double eta_x, int t, double* red) {
  if (mode == 1 && A.scal[DG_S_STATUS] != 0.0) return;
  const double tot = finish_sum(A.partials, A.nblk, red);
  if (threadIdx.x == 0) {
    if (mode == 0)
      *A.div_out = tot / ((double)A.N * (*A.eps));
    else
      div_update_scalars(tot, (double)A.N, *A.eps, A.scal, eta_x, t);
  }
}

__global__ void __launch_bounds__(kRedBlock)
div_kernel(DivArgs A, int mode, uint64_t seed, int iter, double eta_x, int t) {
  __shared__ double red[kRedBlock / 64];
  div_body(A, blockIdx.x, mode, seed, iter, eta_x, t, red);
}
__global__ void __launch_bounds__(kRedBlock)
div_batch(const DivArgs* __restrict__ T, const int* __restrict__ prefix, int n, uint64_t seed,
          int iter, double eta_x, int t) {
  __shared__ double red[kRedBlock / 64];
  const int s = slice_of(prefix, n, blockIdx.x);
  div_body(T[s], blockIdx.x - prefix[s], 1, seed, iter, eta_x, t, red);
}
__global__ void __launch_bounds__(256) div_finish(DivArgs A, int mode, double eta_x, int t) {
  __shared__ double red[4];
  div_finish_body(A, mode, eta_x, t, red);
}
__global__ void __launch_bounds__(256)
div_finish_batch(const DivArgs* __restrict__ T, double eta_x, int t) {
  __shared__ double red[4];
  div_finish_body(T[blockIdx.x], 1, eta_x, t, red);
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
                        float* partials, hipStream_t st) {
  const unsigned int g = red_grid(N);
  hipLaunchKernelGGL(absmax_kernel, dim3(g), dim3(kRedBlock), 0, st, r, N, partials);
  DG_LAUNCH_CHECK("absmax_kernel");
  return launch_eps_finish(partials, (int)g, eps_rel, eps_out, st);
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
    DG_ARG_CHECK(np->patch_radius >= 1 && np->patch_radius <= kMaxP,
                 "denoise: NLM patch radius must be in [1, 3]");
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
  } else if (kind == DG_DEN_TV) {
    return tv_check_params(p, params);
  } else if (kind == DG_DEN_TVW) {
    return tvw_check_params(p, params);
  } else if (kind == DG_DEN_BM3D) {
    return bm3d_check_params(p, params);
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
// NLM with `df` (both images) also performs the divergence step (see NlmArgs).
dg_status launch_denoiser(const dg_plan* p, int kind, const void* params, const float* r,
                          const double* tau_r, const double* eps, uint64_t seed, int iter,
                          float* x_den, float* x_pert, hipStream_t st, const EpsFinish* ef,
                          const DivFuse* df) {
  const int nimg = x_pert ? 2 : 1;
  if (kind == DG_DEN_NLM) {
    const dg_nlm_params* np = (const dg_nlm_params*)params;
    dim3 grid((p->I + kNlmTile - 1) / kNlmTile, (p->I + kNlmTile - 1) / kNlmTile, nimg);
    NlmArgs A{r,       x_den, x_pert, p->I, np->search_radius, tau_r, eps, (float)np->hfac,
              nullptr, 0,     0.0,    nullptr};
    if (ef) {
      A.eps_part = ef->part;
      A.eps_n = ef->n;
      A.eps_rel = ef->eps_rel;
      A.eps_out = ef->out;
    }
    double eta_x = 0.0;
    int t = 0;
    if (df && x_pert) {
      A.x = df->x;
      A.scal = df->scal;
      A.div_part = df->part;
      eta_x = df->eta_x;
      t = df->t;
    }
    nlm_launch(p->nlm_variant, np->patch_radius, grid, st, A, seed, iter, eta_x, t);
    DG_LAUNCH_CHECK("nlm_kernel");
    return DG_OK;
  }
  if (kind == DG_DEN_TV)
    return tv_launch_denoise(p, params, r, tau_r, eps, seed, iter, x_den, x_pert, st);
  if (kind == DG_DEN_TVW)
    return tvw_launch_denoise(p, params, r, tau_r, eps, seed, iter, x_den, x_pert, st);
  if (kind == DG_DEN_BM3D)
    return bm3d_launch_denoise(p, params, r, tau_r, eps, seed, iter, x_den, x_pert, st);
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
                     int iter, double eta_x, int t, double* partials, hipStream_t st) {
  const unsigned int g = red_grid(p->N);
  DivArgs A{p->N, xden, xpert, x, eps, div_out, scal, partials, (int)g};
  hipLaunchKernelGGL(div_kernel, dim3(g), dim3(kRedBlock), 0, st, A, mode, seed, iter, eta_x, t);
  DG_LAUNCH_CHECK("div_kernel");
  hipLaunchKernelGGL(div_finish, dim3(1), dim3(256), 0, st, A, mode, eta_x, t);
  DG_LAUNCH_CHECK("div_finish");
  return DG_OK;
}

// The divergence step's scalar finish (mode 1) alone, one workgroup.
dg_status launch_div_finish(const DivArgs& A, double eta_x, int t, hipStream_t st) {
  hipLaunchKernelGGL(div_finish, dim3(1), dim3(256), 0, st, A, 1, eta_x, t);
  DG_LAUNCH_CHECK("div_finish");
  return DG_OK;
}

unsigned int nlm_blocks(int I) {
  const int g = (I + kNlmTile - 1) / kNlmTile;
  return (unsigned int)(g * g * 2);
}

dg_status launch_nlm_batch(int P, int variant, const NlmArgs* T, const int* prefix, int n,
                           int total, uint64_t seed, int iter, double eta_x, int t,
                           hipStream_t st) {
  if (nlm_waves(variant) == 4)
    nlm_batch_launch_w<4>(P, total, st, T, prefix, n, seed, iter, eta_x, t);
  else
    nlm_batch_launch_w<8>(P, total, st, T, prefix, n, seed, iter, eta_x, t);
  DG_LAUNCH_CHECK("nlm_batch");
  return DG_OK;
}

dg_status launch_div_batch(const DivArgs* T, const int* prefix, int n, int total, uint64_t seed,
                           int iter, double eta_x, int t, hipStream_t st) {
  hipLaunchKernelGGL(div_batch, dim3(total), dim3(kRedBlock), 0, st, T, prefix, n, seed, iter,
                     eta_x, t);
  DG_LAUNCH_CHECK("div_batch");
  hipLaunchKernelGGL(div_finish_batch, dim3(n), dim3(256), 0, st, T, eta_x, t);
  DG_LAUNCH_CHECK("div_finish_batch");
  return DG_OK;
}

// The divergence step's scalar finish alone for n slices (one workgroup each).
dg_status launch_div_finish_batch(const DivArgs* T, int n, double eta_x, int t, hipStream_t st) {
  hipLaunchKernelGGL(div_finish_batch, dim3(n), dim3(256), 0, st, T, eta_x, t);
  DG_LAUNCH_CHECK("div_finish_batch");
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
  float* xpert = nullptr;
  if (div_out) {
    if ((rc = launch_absmax(r, p->N, eps_rel, w.eps, w.fpart, st)) != DG_OK) return rc;
    xpert = w.xpert;
  }
  if (kind == DG_DEN_CNN) {
    rc = cnn_launch_denoise(p, params, r, w.eps, probe_seed, iter, x_out, xpert, nullptr, st);
  } else {
    rc = launch_denoiser(p, kind, params, r, tau_r, w.eps, probe_seed, iter, x_out, xpert, st,
                         nullptr, nullptr);
  }
  if (rc != DG_OK) return rc;
  if (div_out)
    return launch_div(p, x_out, xpert, nullptr, w.eps, div_out, nullptr, 0, probe_seed, iter, 1.0,
                      0, w.dpart, st);
  return DG_OK;
}

// Autotuner of the non-local-means variants on one plan: both are timed on
// r (outputs into out, 2N floats) with fixed tau_r and eps, without the
// divergence step, and the faster is kept.
extern "C" dg_status dg_plan_autotune_nlm(dg_plan* p, const dg_nlm_params* np, const float* r,
                                          float* out, int32_t reps, void* stream) {
  DG_ARG_CHECK(p && np && r && out && reps >= 1, "dg_plan_autotune_nlm: null argument");
  DG_ARG_CHECK(np->patch_radius >= 1 && np->patch_radius <= kMaxP && np->search_radius >= 1 &&
                   np->search_radius <= kMaxS,
               "dg_plan_autotune_nlm: bad NLM parameters");
  hipStream_t st = (hipStream_t)stream;
  double* d = nullptr;
  const double sc[2] = {1e-4, 1e-3};
  DG_HIP(hipMalloc(&d, sizeof(sc)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  dg_status rc = DG_OK;
  if ((e = hipMemcpy(d, sc, sizeof(sc), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
    rc = hip_fail(e, "dg_plan_autotune_nlm");
  const dim3 grid((p->I + kNlmTile - 1) / kNlmTile, (p->I + kNlmTile - 1) / kNlmTile, 2);
  const NlmArgs A{r,       out, out + p->N, p->I, np->search_radius, d, d + 1, (float)np->hfac,
                  nullptr, 0,   0.0,        nullptr};
  float best = 1e30f;
  int best_v = p->nlm_variant;
  for (int v = 0; v < kNlmNumVariants && rc == DG_OK; ++v) {
    nlm_launch(v, np->patch_radius, grid, st, A, 0, 0, 0.0, 0);  // warm
    (void)hipEventRecord(e0, st);
    for (int k = 0; k < reps; ++k) nlm_launch(v, np->patch_radius, grid, st, A, 0, 0, 0.0, 0);
    (void)hipEventRecord(e1, st);
    if ((e = hipGetLastError()) != hipSuccess) {
      rc = hip_fail(e, "dg_plan_autotune_nlm: nlm_kernel");
      break;
    }
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      best_v = v;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(d);
  if (rc == DG_OK) p->nlm_variant = best_v;
  return rc;
}

extern "C" int32_t dg_plan_nlm_variant(const dg_plan* p) { return p ? p->nlm_variant : -1; }

extern "C" dg_status dg_plan_set_nlm_variant(dg_plan* p, int32_t variant) {
  DG_ARG_CHECK(p && variant >= 0 && variant < kNlmNumVariants,
               "dg_plan_set_nlm_variant: bad argument");
  p->nlm_variant = variant;
  return DG_OK;
}
