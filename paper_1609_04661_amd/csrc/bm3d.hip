// Two-stage block-matching 3D collaborative filter (BM3D, Dabov, Foi,
// Katkovnik & Egiazarian 2007), the plug-in denoiser of the paper's
// experiments (Sec. 4.3 treats D as a black box; Sec. 6), and its use in the
// Monte-Carlo divergence (eq. MC_SURE): D(r) and D(r + eps b) in one set of
// launches (grid z = image).
//
//   match   one wavefront per reference block (8 x 8, grid step 3 plus the
//           last position): the 39 x 39 search region in LDS; every lane
//           computes the distances of its candidates (mean squared
//           difference, summed row by row in FP32 without contraction, the
//           order the decisions are defined in); the group is the reference
//           block, then the 15 closest others with d <= 4.8 sigma^2, by
//           (d, raster position), rounded down to a power of two;
//   stage1  one wavefront per group, lane = coefficient (u, v) of an 8 x 8
//           block: 2D DCT of every block (the same fixed FP32 order), Haar
//           pyramid along the group in registers, hard threshold at
//           2.7 sigma, N_har by ballot, inverse transform, aggregation of
//           w K est and w K (w = 1 / (sigma^2 N_har)) by FP32 atomics;
//   basic   y_basic = num / den;
//   stage2  one wavefront per group: transforms of the noisy and the basic
//           blocks, Wiener shrinkage W = T_b^2 / (T_b^2 + sigma^2), weight
//           1 / (sigma^2 ||W||^2) (1 when every factor vanishes), aggregation;
//   final   D = num / den.
// The second stage reuses the first stage's groups, so every decision
// depends on the input alone.  The aggregation sums in FP32 by atomics: the
// result is reproducible to FP32 rounding, not bit for bit.
#include <cmath>

#include "dg_internal.h"

namespace dg {

static constexpr int kB = 8, kB2 = 64, kNs = 19, kN2 = 16, kStep = 3;
static constexpr int kReg = 2 * kNs + kB;  // 46: search region side
static constexpr double kTauMatch = 4.8, kLambda3d = 2.7;
// filter workgroups: a kAggR x kAggR tile of reference positions, whose
// blocks all lie in a kAggW x kAggW pixel tile (positions kStep apart, each
// group's blocks within kNs of its reference, kB pixels each)
static constexpr int kAggR = 4, kAggW = kStep * (kAggR - 1) + 2 * kNs + kB;
static_assert(kAggW == 55, "4 x 4 references span 55 x 55 pixels");

__host__ __device__ inline int bm3d_axis_count(int I) {
  const int n = (I - kB) / kStep + 1;
  return ((n - 1) * kStep == I - kB) ? n : n + 1;
}
__device__ __forceinline__ int bm3d_axis_pos(int a, int I) {
  const int p = a * kStep;
  return p > I - kB ? I - kB : p;
}

struct Bm3dArgs {
  const float* r;       // image 0: the input
  float* rp;            // image 1: r + eps b (formed here)
  float* out0;          // D(r)
  float* out1;          // D(r + eps b) (nullptr: image 0 only)
  int I, na;
  const double* tau_r;
  const double* eps;
  const float* tab;     // DCT matrix (64) and Kaiser window (8)
  int* grp;             // [img][n_ref][kN2]
  int* gsize;           // [img][n_ref]
  float* num;           // [img][N]
  float* den;           // [img][N]
  float* basic;         // [img][N]
};

__device__ __forceinline__ const float* bm3d_in(const Bm3dArgs& A, int img) {
  return img == 0 ? A.r : A.rp;
}

__global__ void __launch_bounds__(256) bm3d_perturb(Bm3dArgs A, uint64_t seed, int iter) {
  const int64_t N = (int64_t)A.I * A.I;
  const float e = (float)(*A.eps);
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < N; k += (int64_t)gridDim.x * 256)
    A.rp[k] = __fadd_rn(A.r[k], e * probe_sign(seed, iter, (uint64_t)k));
}

__global__ void __launch_bounds__(256) bm3d_zero(Bm3dArgs A, int nimg) {
  const int64_t n = (int64_t)nimg * A.I * A.I;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
    A.num[k] = 0.0f;
    A.den[k] = 0.0f;
  }
}

// ---------------------------------------------------------------- matching

// candidates per work item of the matching: a lane takes kRun consecutive
// candidates of one row and slides a kRun + kB - 1 column window of the
// region along each block row
static constexpr int kRun = 5;

__global__ void __launch_bounds__(64) bm3d_match(Bm3dArgs A) {
  // the region, padded so that a run's window may read past the last column
  // (those values feed only candidates past the row's end, which are dropped)
  __shared__ float reg[kReg * kReg + kRun + kB];
  const int img = blockIdx.y;
  const float* r = bm3d_in(A, img);
  const int I = A.I, q = blockIdx.x, lane = threadIdx.x;
  const int yr = bm3d_axis_pos(q / A.na, I), xr = bm3d_axis_pos(q % A.na, I);
  const int ya = max(0, yr - kNs), yb = min(I - kB, yr + kNs);  // candidate rows
  const int xa = max(0, xr - kNs), xb = min(I - kB, xr + kNs);
  const int ry = yb - ya + kB, rx = xb - xa + kB;              // region extent <= 46
  // the region row by row (rx <= 46 < 64: one column per lane)
  for (int y = 0; y < ry; ++y)
    if (lane < rx) reg[y * kReg + lane] = r[(int64_t)(ya + y) * I + xa + lane];
  __syncthreads();
  const float thr = (float)(kTauMatch * *A.tau_r);
  const int ny = yb - ya + 1, nx = xb - xa + 1, nc = ny * nx;
  const int oy = yr - ya, ox = xr - xa;
  // the reference block in registers (the same 64 values in every lane)
  float rv[kB2];
#pragma unroll
  for (int u = 0; u < kB; ++u)
#pragma unroll
    for (int v = 0; v < kB; ++v) rv[u * kB + v] = reg[(oy + u) * kReg + ox + v];
  // each candidate's sum runs over u, then v, each product rounded then
  // added: the same order and roundings as one candidate at a time
  const int runs = (nx + kRun - 1) / kRun;
  // this lane's keys (its work items it = lane + 64 j) and their minimum
  constexpr int kItems = ((2 * kNs + 1) * ((2 * kNs + 1 + kRun - 1) / kRun) + 63) / 64;
  uint64_t lk[kItems][kRun];
  uint64_t lmin = ~0ull;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
#pragma unroll
    for (int k = 0; k < kRun; ++k) lk[j][k] = ~0ull;
    const int it = lane + 64 * j;
    if (it >= ny * runs) continue;
    const int cy = it / runs, cx0 = (it - cy * runs) * kRun;
    float acc[kRun];
#pragma unroll
    for (int k = 0; k < kRun; ++k) acc[k] = 0.0f;
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      float w[kRun + kB - 1];
      const float* rowp = reg + (cy + u) * kReg + cx0;
#pragma unroll
      for (int e = 0; e < kRun + kB - 1; ++e) w[e] = rowp[e];
#pragma unroll
      for (int v = 0; v < kB; ++v)
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
          const float t = __fsub_rn(rv[u * kB + v], w[k + v]);
          acc[k] = __fadd_rn(acc[k], __fmul_rn(t, t));
        }
    }
#pragma unroll
    for (int k = 0; k < kRun; ++k) {
      const int cx = cx0 + k;
      if (cx >= nx) break;
      const float d = __fmul_rn(acc[k], 1.0f / 64.0f);
      const bool self = (cy == oy && cx == ox);
      const uint32_t pos = (uint32_t)((ya + cy) * I + xa + cx);
      const uint64_t key = (d <= thr && !self) ? (((uint64_t)__float_as_uint(d) << 32) | pos) : ~0ull;
      lk[j][k] = key;
      lmin = key < lmin ? key : lmin;
    }
  }
  // the kN2 - 1 smallest keys in ascending order.  Keys are unique (the
  // position is in the low word), so a lane whose minimum is taken finds
  // its next one as the smallest of its own keys above the one taken; the
  // other lanes keep theirs.  Each round: a wavefront minimum over the 64
  // lane minima, and one lane's rescan of its ~25 keys.
  int* g = A.grp + ((int64_t)img * A.na * A.na + q) * kN2;
  int cnt = 1;
  if (lane == 0) g[0] = yr * I + xr;
  for (int k = 1; k < kN2; ++k) {
    uint64_t best = lmin;
    for (int o = 32; o > 0; o >>= 1) {
      const uint64_t other = __shfl_xor(best, o, 64);
      best = other < best ? other : best;
    }
    if (best == ~0ull) break;  // wavefront-uniform
    if (lane == 0) g[k] = (int)(uint32_t)best;
    ++cnt;
    if (lmin == best) {
      uint64_t next = ~0ull;
#pragma unroll
      for (int j = 0; j < kItems; ++j)
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
          const uint64_t key = lk[j][k];
          next = (key > best && key < next) ? key : next;
        }
      lmin = next;
    }
  }
  int p2 = 1;
  while (2 * p2 <= cnt) p2 *= 2;
  if (lane == 0) {
    A.gsize[(int64_t)img * A.na * A.na + q] = p2;
    for (int k = p2; k < kN2; ++k) g[k] = -1;
  }
}

// ---------------------------------------------------------------- transforms

// Orders one wavefront's LDS writes before its later reads of them (and its
// reads before later overwrites): a wavefront's LDS instructions execute in
// issue order, so a wavefront-scope fence and a compiler barrier suffice;
// the wavefronts of a filter workgroup run groups of different sizes, so no
// workgroup barrier may be used here.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 2D DCT of one 8 x 8 block held one value per lane (lane = u * 8 + v),
// T1[u][v] = sum_k D[u][k] B[k][v], C[u][v] = sum_k T1[u][k] D[v][k], each
// product rounded then added, k ascending.
__device__ __forceinline__ float dct2_lane(float bval, const float* D, float* sh) {
  const int lane = threadIdx.x & 63, u = lane >> 3, v = lane & 7;
  sh[lane] = bval;
  wave_lds_sync();
  float acc = 0.0f;
  for (int k = 0; k < kB; ++k) acc = __fadd_rn(acc, __fmul_rn(D[u * kB + k], sh[k * kB + v]));
  wave_lds_sync();
  sh[lane] = acc;
  wave_lds_sync();
  float c = 0.0f;
  for (int k = 0; k < kB; ++k) c = __fadd_rn(c, __fmul_rn(sh[u * kB + k], D[v * kB + k]));
  wave_lds_sync();
  return c;
}

// inverse 2D DCT (any order: continuous)
__device__ __forceinline__ float idct2_lane(float cval, const float* D, float* sh) {
  const int lane = threadIdx.x & 63, u = lane >> 3, v = lane & 7;
  sh[lane] = cval;
  wave_lds_sync();
  float acc = 0.0f;  // T[u][v] = sum_k D[k][u] C[k][v]
  for (int k = 0; k < kB; ++k) acc = __fmaf_rn(D[k * kB + u], sh[k * kB + v], acc);
  wave_lds_sync();
  sh[lane] = acc;
  wave_lds_sync();
  float b = 0.0f;  // B[u][v] = sum_k T[u][k] D[k][v]
  for (int k = 0; k < kB; ++k) b = __fmaf_rn(sh[u * kB + k], D[k * kB + v], b);
  wave_lds_sync();
  return b;
}

// Haar pyramid along a group of NB blocks (a power of two <= 16), one value
// per block in registers: at each level of length L the pairs give
// ((a + b) c, (a - b) c), sums first; c = FP32(1/sqrt 2).
template <int NB>
__device__ __forceinline__ void haar_fwd_g(float (&g)[kN2]) {
  const float c = 0.70710677f;
#pragma unroll
  for (int L = NB; L > 1; L >>= 1) {
    float t[kN2];
#pragma unroll
    for (int i = 0; i < L / 2; ++i) {
      const float a = g[2 * i], b = g[2 * i + 1];
      t[i] = __fmul_rn(__fadd_rn(a, b), c);
      t[L / 2 + i] = __fmul_rn(__fsub_rn(a, b), c);
    }
#pragma unroll
    for (int i = 0; i < L; ++i) g[i] = t[i];
  }
}
template <int NB>
__device__ __forceinline__ void haar_inv_g(float (&g)[kN2]) {
  const float c = 0.70710677f;
#pragma unroll
  for (int L = 2; L <= NB; L <<= 1) {
    float t[kN2];
#pragma unroll
    for (int i = 0; i < L / 2; ++i) {
      const float a = g[i], d = g[L / 2 + i];
      t[2 * i] = (a + d) * c;
      t[2 * i + 1] = (a - d) * c;
    }
#pragma unroll
    for (int i = 0; i < L; ++i) g[i] = t[i];
  }
}

__device__ __forceinline__ float wave_sum_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------- stages

// One group of NB blocks (lane = coefficient (u, v)); g: its block positions.
template <int STAGE, int NB>
__device__ void bm3d_group(const Bm3dArgs& A, int img, const int* g, const float* D, const float* K,
                           float* sh, float* snum, float* sden, int y0, int x0) {
  const int lane = threadIdx.x & 63, u = lane >> 3, v = lane & 7;
  const int I = A.I;
  const int64_t N = (int64_t)I * I;
  const float* r = bm3d_in(A, img);
  const double s2 = *A.tau_r;
  float tn[kN2], tb[kN2];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int p = g[b];
    const int64_t off = (int64_t)(p / I + u) * I + p % I + v;
    tn[b] = dct2_lane(r[off], D, sh);
    if (STAGE == 2) tb[b] = dct2_lane(A.basic[img * N + off], D, sh);
  }
  haar_fwd_g<NB>(tn);
  float w;
  if (STAGE == 1) {
    const float thr = (float)(kLambda3d * sqrt(s2));
    int kept = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const bool keep = fabsf(tn[b]) > thr;
      if (!keep) tn[b] = 0.0f;
      kept += __popcll(__ballot(keep));
    }
    w = kept >= 1 ? (float)(1.0 / (s2 * (double)kept)) : 1.0f;
  } else {
    haar_fwd_g<NB>(tb);
    float wsq = 0.0f;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const float t2 = tb[b] * tb[b];
      const float W = t2 / (t2 + (float)s2);
      tn[b] *= W;
      wsq += W * W;
    }
    wsq = wave_sum_f(wsq);
    // a group on which the basic estimate vanishes has W = 0: weight 1, the
    // first stage's rule for a group without surviving coefficients
    w = wsq > 0.0f ? (float)(1.0 / (s2 * (double)wsq)) : 1.0f;
  }
  haar_inv_g<NB>(tn);
  const float wk = w * K[u] * K[v];
  float* num = A.num + img * N;
  float* den = A.den + img * N;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const float est = idct2_lane(tn[b], D, sh);
    const int p = g[b];
    const int py = p / I + u, px = p % I + v;
    // the workgroup's tile of sums in LDS (every block of its groups lies
    // inside it; the global fallback only guards the indexing)
    const int ly = py - y0, lx = px - x0;
    if (snum && (unsigned)ly < (unsigned)kAggW && (unsigned)lx < (unsigned)kAggW) {
      atomicAdd(snum + ly * kAggW + lx, wk * est);
      atomicAdd(sden + ly * kAggW + lx, wk);
    } else {
      const int64_t off = (int64_t)py * I + px;
      atomicAdd(num + off, wk * est);
      atomicAdd(den + off, wk);
    }
  }
}

// Stage-1 filter: a workgroup filters the groups of a kAggR x kAggR tile of
// reference positions, kAggR^2 / 4 per wavefront, adding their weighted
// estimates into a kAggW x kAggW tile of num and den in LDS (LDS atomics);
// the tile then goes to the image's accumulators with one global atomic per
// pixel and sum, about a fifth as many as adding every block's pixels there
// (1.12 -> 0.82 ms per call at 512^2).  The Wiener stage keeps one group per
// single-wavefront workgroup (bm3d_filter_group): at 322 VGPRs a 4-wavefront
// workgroup holds a whole compute unit until its slowest group is done, and
// the tiled form ran slower there (1.43 -> 1.53 ms).  The sums' order is
// unspecified either way (FP32 atomics).
template <int STAGE>
__global__ void __launch_bounds__(256) bm3d_filter(Bm3dArgs A) {
  __shared__ float snum[kAggW * kAggW], sden[kAggW * kAggW];
  __shared__ float sh[4][kB2];
  __shared__ float D[kB2];
  __shared__ float K[kB];
  const int img = blockIdx.y, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int I = A.I, na = A.na;
  const int tiles = (na + kAggR - 1) / kAggR;
  const int tqy = (blockIdx.x / tiles) * kAggR, tqx = (blockIdx.x % tiles) * kAggR;
  // the tile's origin: its first reference position less the search
  // radius (blocks start at most kNs before their reference)
  const int y0 = max(0, bm3d_axis_pos(tqy, I) - kNs), x0 = max(0, bm3d_axis_pos(tqx, I) - kNs);
  for (int e = threadIdx.x; e < kAggW * kAggW; e += 256) snum[e] = sden[e] = 0.0f;
  if (threadIdx.x < kB2) D[threadIdx.x] = A.tab[threadIdx.x];
  if (threadIdx.x < kB) K[threadIdx.x] = A.tab[kB2 + threadIdx.x];
  __syncthreads();
  const int nref = na * na;
  for (int e = wave; e < kAggR * kAggR; e += 4) {
    const int qy = tqy + e / kAggR, qx = tqx + e % kAggR;
    if (qy >= na || qx >= na) continue;  // wavefront-uniform
    const int q = qy * na + qx;
    const int* g = A.grp + ((int64_t)img * nref + q) * kN2;
    switch (A.gsize[(int64_t)img * nref + q]) {  // uniform per wavefront
      case 16: bm3d_group<STAGE, 16>(A, img, g, D, K, sh[wave], snum, sden, y0, x0); break;
      case 8: bm3d_group<STAGE, 8>(A, img, g, D, K, sh[wave], snum, sden, y0, x0); break;
      case 4: bm3d_group<STAGE, 4>(A, img, g, D, K, sh[wave], snum, sden, y0, x0); break;
      case 2: bm3d_group<STAGE, 2>(A, img, g, D, K, sh[wave], snum, sden, y0, x0); break;
      default: bm3d_group<STAGE, 1>(A, img, g, D, K, sh[wave], snum, sden, y0, x0); break;
    }
  }
  __syncthreads();
  const int64_t N = (int64_t)I * I;
  float* num = A.num + img * N;
  float* den = A.den + img * N;
  for (int e = threadIdx.x; e < kAggW * kAggW; e += 256) {
    const int py = y0 + e / kAggW, px = x0 + e % kAggW;
    const float dv = sden[e];
    if (py < I && px < I && dv != 0.0f) {
      atomicAdd(num + (int64_t)py * I + px, snum[e]);
      atomicAdd(den + (int64_t)py * I + px, dv);
    }
  }
}

// One group per single-wavefront workgroup, its estimates added straight
// into the image's accumulators.
template <int STAGE>
__global__ void __launch_bounds__(64) bm3d_filter_group(Bm3dArgs A) {
  __shared__ float sh[kB2];
  __shared__ float D[kB2];
  __shared__ float K[kB];
  const int img = blockIdx.y, q = blockIdx.x, lane = threadIdx.x;
  D[lane] = A.tab[lane];
  if (lane < kB) K[lane] = A.tab[kB2 + lane];
  __syncthreads();
  const int nref = A.na * A.na;
  const int* g = A.grp + ((int64_t)img * nref + q) * kN2;
  switch (A.gsize[(int64_t)img * nref + q]) {  // uniform per workgroup
    case 16: bm3d_group<STAGE, 16>(A, img, g, D, K, sh, nullptr, nullptr, 0, 0); break;
    case 8: bm3d_group<STAGE, 8>(A, img, g, D, K, sh, nullptr, nullptr, 0, 0); break;
    case 4: bm3d_group<STAGE, 4>(A, img, g, D, K, sh, nullptr, nullptr, 0, 0); break;
    case 2: bm3d_group<STAGE, 2>(A, img, g, D, K, sh, nullptr, nullptr, 0, 0); break;
    default: bm3d_group<STAGE, 1>(A, img, g, D, K, sh, nullptr, nullptr, 0, 0); break;
  }
}

// basic (STAGE 1) or final output (STAGE 2) = num / den; the accumulators are
// cleared for the next stage.
template <int STAGE>
__global__ void __launch_bounds__(256) bm3d_divide(Bm3dArgs A, int nimg) {
  const int64_t N = (int64_t)A.I * A.I;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nimg * N; k += (int64_t)gridDim.x * 256) {
    const float v = A.num[k] / A.den[k];
    if (STAGE == 1) {
      A.basic[k] = v;
      A.num[k] = 0.0f;
      A.den[k] = 0.0f;
    } else {
      (k < N ? A.out0[k] : A.out1[k - N]) = v;
    }
  }
}

static size_t bm3d_layout(int I, void* base, Bm3dArgs* A) {
  char* c = (char*)base;
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = c ? c + off : nullptr;
    off += (b + 255) & ~(size_t)255;
    return q;
  };
  const int na = bm3d_axis_count(I);
  const size_t N = (size_t)I * I, nref = (size_t)na * na;
  Bm3dArgs t{};
  t.na = na;
  t.rp = (float*)take(sizeof(float) * N);
  t.grp = (int*)take(sizeof(int) * 2 * nref * kN2);
  t.gsize = (int*)take(sizeof(int) * 2 * nref);
  t.num = (float*)take(sizeof(float) * 2 * N);
  t.den = (float*)take(sizeof(float) * 2 * N);
  t.basic = (float*)take(sizeof(float) * 2 * N);
  if (A) *A = t;
  return off;
}

size_t bm3d_work_bytes(int I) { return I >= kB ? bm3d_layout(I, nullptr, nullptr) : 0; }

dg_status bm3d_check_params(const dg_plan* p, const void* params) {
  DG_ARG_CHECK(params != nullptr, "denoise: BM3D params must not be NULL");
  DG_ARG_CHECK(((const dg_bm3d_params*)params)->work != nullptr, "denoise: BM3D work must not be NULL");
  DG_ARG_CHECK(p->I >= 16 && p->I <= 4096, "denoise: BM3D needs 16 <= I <= 4096");
  return DG_OK;
}

dg_status bm3d_launch_denoise(const dg_plan* p, const void* params, const float* r,
                              const double* tau_r, const double* eps, uint64_t seed, int iter,
                              float* x_den, float* x_pert, hipStream_t st) {
  const dg_bm3d_params* bp = (const dg_bm3d_params*)params;
  Bm3dArgs A;
  bm3d_layout(p->I, bp->work, &A);
  A.r = r;
  A.out0 = x_den;
  A.out1 = x_pert;
  A.I = p->I;
  A.tau_r = tau_r;
  A.eps = eps;
  A.tab = p->bm3d_tab;
  const int nimg = x_pert ? 2 : 1;
  const int nref = A.na * A.na;
  const unsigned int ge = grid_for((int64_t)nimg * p->N, 256, 4096);
  if (x_pert) {
    hipLaunchKernelGGL(bm3d_perturb, dim3(grid_for(p->N, 256, 4096)), dim3(256), 0, st, A, seed, iter);
    DG_LAUNCH_CHECK("bm3d_perturb");
  }
  hipLaunchKernelGGL(bm3d_zero, dim3(ge), dim3(256), 0, st, A, nimg);
  DG_LAUNCH_CHECK("bm3d_zero");
  hipLaunchKernelGGL(bm3d_match, dim3(nref, nimg), dim3(64), 0, st, A);
  DG_LAUNCH_CHECK("bm3d_match");
  const int tiles = (A.na + kAggR - 1) / kAggR;
  hipLaunchKernelGGL(bm3d_filter<1>, dim3(tiles * tiles, nimg), dim3(256), 0, st, A);
  DG_LAUNCH_CHECK("bm3d_filter<1>");
  hipLaunchKernelGGL(bm3d_divide<1>, dim3(ge), dim3(256), 0, st, A, nimg);
  DG_LAUNCH_CHECK("bm3d_divide<1>");
  hipLaunchKernelGGL(bm3d_filter_group<2>, dim3(nref, nimg), dim3(64), 0, st, A);
  DG_LAUNCH_CHECK("bm3d_filter_group<2>");
  hipLaunchKernelGGL(bm3d_divide<2>, dim3(ge), dim3(256), 0, st, A, nimg);
  DG_LAUNCH_CHECK("bm3d_divide<2>");
  return DG_OK;
}

}  // namespace dg

extern "C" size_t dg_bm3d_workspace_bytes(int32_t side) { return dg::bm3d_work_bytes(side); }
