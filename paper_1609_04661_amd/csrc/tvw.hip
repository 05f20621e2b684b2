// Proximal total variation in the (V^T V)^-1 metric (Sec. 4.3 and Sec. 6
// name it for input in the preconditioned domain; Sec. 4.3 treats D as a
// black box):
//   D(r) = argmin_x 1/2 (x - r)^T W (x - r) + lam TV(x),  W = (V^T V)^-1,
// lam = alpha sqrt(tau_r), W circulant with symbol w = 1/c (c the cone
// symbol: |k| / I off DC, 1 / (4 ln(1 + sqrt 2) I) at DC).  The paper's
// figure writes the subscript V^T V instead; that reading (w = c) is the
// `metric` switch.  Either weight spans three orders of magnitude over the
// grid, so unlike the l2 map no dual-only method is practical (its step
// would scale with 1/min w); K Chambolle-Pock steps
// (Chambolle & Pock 2011, theta = 1) with the operator lam grad and
// sigma = tau = 1 / (lam sqrt 8):
//   p    = P(p + grad(xbar) / sqrt 8)                 (sigma lam = 1/sqrt 8)
//   v    = x - grad^T(p) / sqrt 8                     (tau lam = 1/sqrt 8)
//   x'   = F^-1 [(F v + tau w F r) / (1 + tau w)]     (the primal prox of G)
//   xbar = 2 x' - x
// from x = xbar = r, p = 0; the map is those K steps.  Each step is three
// launches over both images (r and the probe's r + eps b), the passes of a
// 2D FFT solve: row transforms of v, with the dual update fused in front
// (a row pair's v needs the new dual on its rows and on the row above; the
// dual is ping-ponged between two buffers so that the rows recomputed by a
// neighbouring workgroup still read the old one), column transforms with the
// Fourier-domain division, inverse row transforms with the extrapolation.
// F r is computed once per call.  The FFT passes share the wavefront
// transforms of the cone preconditioner.
#include <cmath>
#include <utility>

#include "dg_internal.h"
#include "fft_wave.h"

namespace dg {

struct TvwArgs {
  const float* r;       // image 0 input
  float* b1;            // image 1 input r + eps b (written by tvw_prep)
  float* x;             // primal, [img][N]
  float* xb;            // extrapolated primal, [img][N]
  float* p;             // dual read by a step, [img][2][N]
  float* pn;            // dual written by a step, [img][2][N] (swapped with p per step)
  float2* spec;         // [img][spec_n]: row-transformed / solved spectrum, spec[k][row]
  float2* rspec;        // [img][spec_n]: F r, after the column transforms
  const float2* tw;     // plan twiddles, I entries
  int I;
  int nimg;
  int metric;           // 0: w = 1/c, 1: w = c
  float alpha;
  const double* tau_r;
  const double* eps;
  float* out0;
  float* out1;
  int64_t npix;         // I * I
  int64_t N;            // plane stride (npix rounded up to 256 bytes)
  int64_t spec_n;       // spectrum stride ((I/2 + 1) I rounded up to 256 bytes)
};

static constexpr float kInvSqrt8 = 0.35355339059327376220f;

// tau = 1 / (lam sqrt 8), 0 when lam = 0 (then every step keeps x = r).
__device__ __forceinline__ float tvw_tau(const TvwArgs& A) {
  const double t = *A.tau_r;
  const float lam = t > 0.0 ? A.alpha * (float)sqrt(t) : 0.0f;
  return lam > 0.0f ? kInvSqrt8 / lam : 0.0f;
}
__device__ __forceinline__ const float* tvw_input(const TvwArgs& A, int img) {
  return img ? A.b1 : A.r;
}

// b1 = r + eps b; x = xbar = input; p = 0.
__global__ void __launch_bounds__(256) tvw_prep(TvwArgs A, uint64_t seed, int iter) {
  const float eps = A.nimg > 1 ? (float)(*A.eps) : 0.0f;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < A.npix;
       k += (int64_t)gridDim.x * blockDim.x) {
    const float r = A.r[k];
    const float b1 = __fmaf_rn(eps, probe_sign(seed, iter, (uint64_t)k), r);
    if (A.nimg > 1) A.b1[k] = b1;
    for (int m = 0; m < A.nimg; ++m) {
      const float b = m ? b1 : r;
      A.x[m * A.N + k] = b;
      A.xb[m * A.N + k] = b;
      A.p[(2 * m) * A.N + k] = 0.0f;
      A.p[(2 * m + 1) * A.N + k] = 0.0f;
    }
  }
}

// The new dual at (a, b): P(p + sl grad(xbar)), forward differences with
// zero past the last row / column, P the projection onto the unit disc.
__device__ __forceinline__ float2 tvw_pnew(const float* __restrict__ xb, const float* __restrict__ p1,
                                           const float* __restrict__ p2, int a, int b, int I,
                                           float sl) {
  const int64_t k = (int64_t)a * I + b;
  const float c = xb[k];
  const float g1 = a < I - 1 ? xb[k + I] - c : 0.0f;
  const float g2 = b < I - 1 ? xb[k + 1] - c : 0.0f;
  const float q1 = __fmaf_rn(sl, g1, p1[k]);
  const float q2 = __fmaf_rn(sl, g2, p2[k]);
  const float inv = 1.0f / fmaxf(1.0f, sqrtf(__fmaf_rn(q1, q1, q2 * q2)));
  return make_float2(q1 * inv, q2 * inv);
}

// Row pass: workgroup blockIdx.x owns real rows kRowsPerBlock blk onwards of
// image blockIdx.y; mode 0 transforms the input, mode 1 first takes the
// dual step p' = P(p + grad(xbar) / sqrt 8) on its rows (written to pn) and
// transforms v = x - grad^T(p') / sqrt 8; the adjoint's p' on the row above
// is recomputed, the one a column to the left is taken from the neighbouring
// lane.  Output
// spec[k][row], k = 0..I/2, as the cone preconditioner's row pass.
__global__ void __launch_bounds__(kFftThreads) tvw_rows(TvwArgs A, int mode) {
  __shared__ FftShared S;
  const int I = A.I, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int blk = blockIdx.x, img = blockIdx.y;
  const int half = I / 2 + 1;
  const int m = blk * kFftWaves + w;
  const bool live = 2 * m < I;
  const float* src = mode ? A.x + img * A.N : tvw_input(A, img);
  const float* xbar = A.xb + img * A.N;
  const float* p1 = A.p + (2 * img) * A.N;
  const float* p2 = p1 + A.N;
  float* q1 = A.pn + (2 * img) * A.N;
  float* q2 = q1 + A.N;
  float2* spec = A.spec + img * A.spec_n;
  // sigma lam = tau lam = 1/sqrt 8; 0 when lam = 0 (the identity map)
  const float sl = tvw_tau(A) > 0.0f ? kInvSqrt8 : 0.0f;
  float ra[kPerLane], rb[kPerLane];
  if (live) {
    const int ia = 2 * m, ib = 2 * m + 1;
    // p2' one column to the left comes from the neighbouring lane, and for
    // lane 0 from lane 63 of the previous group of 64 columns
    float carry_a = 0.0f, carry_b = 0.0f;
#pragma unroll
    for (int q = 0; q < kPerLane; ++q) {
      const int t = lane + 64 * q;
      if (64 * q < I) {  // wavefront-uniform: the shuffles need every lane
        const bool in = t < I;
        float va = in ? src[(int64_t)ia * I + t] : 0.0f;
        float vb = in ? src[(int64_t)ib * I + t] : 0.0f;
        if (mode) {
          float2 na = make_float2(0.0f, 0.0f), nb = na, nu = na;
          if (in) {
            na = tvw_pnew(xbar, p1, p2, ia, t, I, sl);
            nb = tvw_pnew(xbar, p1, p2, ib, t, I, sl);
            if (ia > 0) nu = tvw_pnew(xbar, p1, p2, ia - 1, t, I, sl);  // the row above
            q1[(int64_t)ia * I + t] = na.x;
            q2[(int64_t)ia * I + t] = na.y;
            q1[(int64_t)ib * I + t] = nb.x;
            q2[(int64_t)ib * I + t] = nb.y;
          }
          float la = __shfl_up(na.y, 1, 64), lb = __shfl_up(nb.y, 1, 64);
          if (lane == 0) {
            la = carry_a;
            lb = carry_b;
          }
          carry_a = __shfl(na.y, 63, 64);
          carry_b = __shfl(nb.y, 63, 64);
          // grad^T p' in the order of the adjoint's terms: +p1(i-1), -p1(i),
          // +p2(j-1), -p2(j)
          float aa = 0.0f, ab = 0.0f;
          if (ia > 0) aa += nu.x;
          aa -= na.x;  // ia < I - 1 always (ib = ia + 1 exists)
          if (t > 0) aa += la;
          if (t < I - 1) aa -= na.y;
          ab += na.x;  // ib > 0
          if (ib < I - 1) ab -= nb.x;
          if (t > 0) ab += lb;
          if (t < I - 1) ab -= nb.y;
          va = __fmaf_rn(-sl, aa, va);
          vb = __fmaf_rn(-sl, ab, vb);
        }
        ra[q] = va;
        rb[q] = vb;
      }
    }
  }
  float2* a = S.buf[w][0];
  float2* b = S.buf[w][1];
  if (I == 512 || I == 256) {
    if (live) {
      if (I == 512)
        rows_fwd_reg<8, 3>(A.tw, ra, rb, a, b);
      else
        rows_fwd_reg<4, 4>(A.tw, ra, rb, a, b);
    }
  } else {
    load_twiddles(S, A.tw, I);
    if (live) {
#pragma unroll
      for (int q = 0; q < kPerLane; ++q) {
        const int t = lane + 64 * q;
        if (t < I) a[t] = make_float2(ra[q], rb[q]);
      }
      wave_sync();
      wave_fft(a, b, I, S.tw, false);
    }
  }
  if (live) {
    for (int k = lane; k < half; k += 64) {
      float2 Z = a[k], Zc = a[(I - k) % I];
      Zc.y = -Zc.y;
      float2 Xa = make_float2(0.5f * (Z.x + Zc.x), 0.5f * (Z.y + Zc.y));
      float2 d = make_float2(0.5f * (Z.x - Zc.x), 0.5f * (Z.y - Zc.y));
      b[k] = Xa;
      b[half + k] = make_float2(d.y, -d.x);  // d / i
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < half * kRowsPerBlock; idx += blockDim.x) {
    const int k = idx / kRowsPerBlock, c = idx % kRowsPerBlock;
    const int row = blk * kRowsPerBlock + c;
    if (row < I) spec[(int64_t)k * I + row] = S.buf[c >> 1][1][(c & 1) * half + k];
  }
}

// Column pass: wavefront w of workgroup blockIdx.x takes column frequency
// kx = kFftWaves blk + w of image blockIdx.y.  Mode 0 stores the column
// transform as F r (rspec); mode 1 solves (1 + tau w) X = V + tau w R per
// frequency and transforms back in place.
__global__ void __launch_bounds__(kFftThreads) tvw_cols(TvwArgs A, int mode) {
  __shared__ FftShared S;
  const int I = A.I, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int img = blockIdx.y;
  const int kx = blockIdx.x * kFftWaves + w;
  const bool live = kx <= I / 2;
  float2* col = A.spec + img * A.spec_n + (int64_t)kx * I;
  const float2* rcol = A.rspec + img * A.spec_n + (int64_t)kx * I;
  float2* rcol_w = A.rspec + img * A.spec_n + (int64_t)kx * I;
  const float tau = mode ? tvw_tau(A) : 0.0f;
  const float dc = 3.52549435174692f * (float)I;  // 4 ln(1 + sqrt 2) I
  // w at (kx, t): 1/c = |k| / I off DC (metric 0) or c = I / |k| (metric 1)
  auto metric = [&](int t) {
    const int ky = (t <= I / 2) ? t : t - I;
    const float k2 = (float)(kx * kx + ky * ky);
    if (A.metric) return k2 > 0.0f ? (float)I / sqrtf(k2) : dc;
    return k2 > 0.0f ? sqrtf(k2) / (float)I : 1.0f / dc;
  };
  float2 cv[kPerLane];
  if (live) {
#pragma unroll
    for (int q = 0; q < kPerLane; ++q) {
      const int t = lane + 64 * q;
      if (t < I) cv[q] = col[t];
    }
  }
  float2* a = S.buf[w][0];
  float2* b = S.buf[w][1];
  const bool reg = I == 512 || I == 256;
  if (!reg) load_twiddles(S, A.tw, I);
  if (!live) return;
  auto solve = [&](int t, float2 v) {
    const float2 R = rcol[t];
    const float s = tau * metric(t);
    const float inv = 1.0f / (1.0f + s);
    return make_float2(__fmaf_rn(s, R.x, v.x) * inv, __fmaf_rn(s, R.y, v.y) * inv);
  };
  if (reg) {
    if (I == 512) {
      RegTw<8, 3> T;
      reg_tw_load(T, A.tw);
      float2 v[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = cv[r];
      reg_fft<8, 3>(v, T, reinterpret_cast<float*>(a), false);
      if (mode == 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r) rcol_w[lane + 64 * r] = v[r];
        return;
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = solve(lane + 64 * r, v[r]);
      reg_fft<8, 3>(v, T, reinterpret_cast<float*>(a), true);
#pragma unroll
      for (int r = 0; r < 8; ++r) col[lane + 64 * r] = v[r];
    } else {
      RegTw<4, 4> T;
      reg_tw_load(T, A.tw);
      float2 v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = cv[r];
      reg_fft<4, 4>(v, T, reinterpret_cast<float*>(a), false);
      if (mode == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) rcol_w[lane + 64 * r] = v[r];
        return;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = solve(lane + 64 * r, v[r]);
      reg_fft<4, 4>(v, T, reinterpret_cast<float*>(a), true);
#pragma unroll
      for (int r = 0; r < 4; ++r) col[lane + 64 * r] = v[r];
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < kPerLane; ++q) {
    const int t = lane + 64 * q;
    if (t < I) a[t] = cv[q];
  }
  wave_sync();
  wave_fft(a, b, I, S.tw, false);
  if (mode == 0) {
    for (int t = lane; t < I; t += 64) rcol_w[t] = a[t];
    return;
  }
  for (int t = lane; t < I; t += 64) a[t] = solve(t, a[t]);
  wave_sync();
  wave_fft(a, b, I, S.tw, true);
  for (int t = lane; t < I; t += 64) col[t] = a[t];
}

// Inverse row pass: x' = F^-1 (solved spectrum) for the rows of workgroup
// blockIdx.x of image blockIdx.y; xbar = 2 x' - x, x = x'.  On the last
// step x' goes to the output instead.
__global__ void __launch_bounds__(kFftThreads) tvw_rows_inv(TvwArgs A, int last) {
  __shared__ FftShared S;
  const int I = A.I, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int blk = blockIdx.x, img = blockIdx.y;
  const int half = I / 2 + 1;
  const int m = blk * kFftWaves + w;
  const bool live = 2 * m < I;
  const bool reg = I == 512 || I == 256;
  const float2* spec = A.spec + img * A.spec_n;
  float* x = A.x + img * A.N;
  float* xb = A.xb + img * A.N;
  float* out = img ? A.out1 : A.out0;
  const float* in = tvw_input(A, img);
  const bool ident = !(tvw_tau(A) > 0.0f);  // lam = 0: D is the identity
  constexpr int kSpecPer = (kMaxFft / 2 + 1) * kRowsPerBlock / kFftThreads + 1;
  float2 sv[kSpecPer];
#pragma unroll
  for (int q = 0; q < kSpecPer; ++q) {
    const int idx = threadIdx.x + kFftThreads * q;
    const int k = idx / kRowsPerBlock, c = idx % kRowsPerBlock;
    const int row = blk * kRowsPerBlock + c;
    sv[q] = make_float2(0.0f, 0.0f);
    if (idx < half * kRowsPerBlock && row < I) sv[q] = spec[(int64_t)k * I + row];
  }
  if (!reg) load_twiddles(S, A.tw, I);
#pragma unroll
  for (int q = 0; q < kSpecPer; ++q) {
    const int idx = threadIdx.x + kFftThreads * q;
    const int k = idx / kRowsPerBlock, c = idx % kRowsPerBlock;
    if (idx < half * kRowsPerBlock) S.buf[c >> 1][1][(c & 1) * half + k] = sv[q];
  }
  __syncthreads();
  if (!live) return;
  float2* a = S.buf[w][0];
  float2* b = S.buf[w][1];
  const float scale = 1.0f / ((float)I * (float)I);
  auto pair = [&](int t) {
    float2 ya, yb;
    if (t < half) {
      ya = b[t];
      yb = b[half + t];
    } else {
      ya = b[I - t];
      yb = b[half + I - t];
      ya.y = -ya.y;
      yb.y = -yb.y;
    }
    return make_float2(ya.x - yb.y, ya.y + yb.x);
  };
  auto emit = [&](int, int t, float2 z) {
    const int64_t i0 = (int64_t)(2 * m) * I + t, i1 = i0 + I;
    const float v0 = z.x * scale, v1 = z.y * scale;
    if (last) {
      out[i0] = ident ? in[i0] : v0;
      out[i1] = ident ? in[i1] : v1;
    } else {
      const float o0 = x[i0], o1 = x[i1];
      x[i0] = v0;
      x[i1] = v1;
      xb[i0] = __fmaf_rn(2.0f, v0, -o0);
      xb[i1] = __fmaf_rn(2.0f, v1, -o1);
    }
  };
  if (I == 512) {
    rows_inv_reg<8, 3>(A.tw, pair, emit, reinterpret_cast<float*>(a));
  } else if (I == 256) {
    rows_inv_reg<4, 4>(A.tw, pair, emit, reinterpret_cast<float*>(a));
  } else {
    for (int t = lane; t < I; t += 64) a[t] = pair(t);
    wave_sync();
    wave_fft(a, b, I, S.tw, true);
    for (int t = lane; t < I; t += 64) emit(0, t, a[t]);
  }
}

static size_t tvw_align(size_t n) { return (n + 255) & ~(size_t)255; }

size_t tvw_work_bytes(int64_t npix, int I) {
  // b1; x, xb for two images; p and pn (2 components each) for two images;
  // spec and rspec for two images
  const size_t f = tvw_align(sizeof(float) * (size_t)npix);
  const size_t sp = tvw_align(sizeof(float2) * (size_t)(I / 2 + 1) * (size_t)I);
  return f + 2 * 2 * f + 2 * 2 * 2 * f + 2 * 2 * sp;
}

dg_status tvw_check_params(const dg_plan* p, const void* params) {
  DG_ARG_CHECK(params != nullptr, "denoise: TVW params must not be NULL");
  const dg_tv_params* tp = (const dg_tv_params*)params;
  DG_ARG_CHECK(tp->alpha >= 0 && std::isfinite(tp->alpha), "denoise: TVW alpha must be >= 0");
  DG_ARG_CHECK(tp->iters >= 1 && tp->iters <= 10000, "denoise: TVW iters must be in [1, 10000]");
  DG_ARG_CHECK(tp->work != nullptr, "denoise: TVW work buffer must not be NULL");
  DG_ARG_CHECK(tp->metric == 0 || tp->metric == 1, "denoise: TVW metric must be 0 or 1");
  DG_ARG_CHECK(p->fft_ok && p->twiddle != nullptr,
               "denoise: TVW needs an image side the FFT supports (2^a or 3*2^a, <= 1024)");
  return DG_OK;
}

dg_status tvw_launch_denoise(const dg_plan* p, const void* params, const float* r,
                             const double* tau_r, const double* eps, uint64_t seed, int iter,
                             float* x_den, float* x_pert, hipStream_t st) {
  const dg_tv_params* tp = (const dg_tv_params*)params;
  const int I = p->I;
  const int64_t N = (int64_t)I * I;
  const size_t f = tvw_align(sizeof(float) * (size_t)N);
  const size_t sp = tvw_align(sizeof(float2) * (size_t)(I / 2 + 1) * (size_t)I);
  char* c = (char*)tp->work;
  TvwArgs A;
  A.r = r;
  A.b1 = (float*)c;
  A.x = (float*)(c + f);        // 2 planes, f apart
  A.xb = (float*)(c + 3 * f);   // 2 planes
  A.p = (float*)(c + 5 * f);    // 4 planes
  A.pn = (float*)(c + 9 * f);   // 4 planes
  A.spec = (float2*)(c + 13 * f);          // 2 spectra, sp apart
  A.rspec = (float2*)(c + 13 * f + 2 * sp);
  A.tw = p->twiddle;
  A.I = I;
  A.nimg = x_pert ? 2 : 1;
  A.metric = tp->metric;
  A.alpha = (float)tp->alpha;
  A.tau_r = tau_r;
  A.eps = eps;
  A.out0 = x_den;
  A.out1 = x_pert;
  // plane and spectrum strides in elements (the regions are padded to 256 B)
  A.npix = N;
  A.N = (int64_t)(f / sizeof(float));
  A.spec_n = (int64_t)(sp / sizeof(float2));
  const unsigned int g = (unsigned int)((N + 255) / 256 < 2048 ? (N + 255) / 256 : 2048);
  // the kernels index planes A.N floats apart and touch only the first I*I of each
  TvwArgs K = A;
  hipLaunchKernelGGL(tvw_prep, dim3(g), dim3(256), 0, st, K, seed, iter);
  DG_LAUNCH_CHECK("tvw_prep");
  const dim3 rgrid((I + kRowsPerBlock - 1) / kRowsPerBlock, A.nimg);
  const dim3 cgrid((I / 2 + 1 + kFftWaves - 1) / kFftWaves, A.nimg);
  hipLaunchKernelGGL(tvw_rows, rgrid, dim3(kFftThreads), 0, st, K, 0);
  DG_LAUNCH_CHECK("tvw_rows");
  hipLaunchKernelGGL(tvw_cols, cgrid, dim3(kFftThreads), 0, st, K, 0);
  DG_LAUNCH_CHECK("tvw_cols");
  for (int k = 0; k < tp->iters; ++k) {
    if (k > 0) std::swap(K.p, K.pn);  // this step reads the dual the last one wrote
    hipLaunchKernelGGL(tvw_rows, rgrid, dim3(kFftThreads), 0, st, K, 1);
    DG_LAUNCH_CHECK("tvw_rows");
    hipLaunchKernelGGL(tvw_cols, cgrid, dim3(kFftThreads), 0, st, K, 1);
    DG_LAUNCH_CHECK("tvw_cols");
    hipLaunchKernelGGL(tvw_rows_inv, rgrid, dim3(kFftThreads), 0, st, K,
                       k + 1 == tp->iters ? 1 : 0);
    DG_LAUNCH_CHECK("tvw_rows_inv");
  }
  return DG_OK;
}

}  // namespace dg

using namespace dg;

extern "C" size_t dg_tvw_workspace_bytes(int32_t side) {
  return side > 0 ? tvw_work_bytes((int64_t)side * side, side) : 0;
}
