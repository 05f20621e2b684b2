// Wavefront FFT building blocks shared by the cone preconditioner and the
// (V^T V)^-1-metric proximal TV: one complex transform of length L <= 1024
// per wavefront, as a Stockham autosort transform either held in registers
// (L = 512 and 256) or staged through LDS (other lengths), with twiddles
// from a table exp(-2 pi i j / L) computed in FP64 at plan time.
#pragma once

#include "dg_internal.h"

namespace dg {

static constexpr int kFftWaves = 4;                 // one FFT per wavefront
static constexpr int kFftThreads = 64 * kFftWaves;
static constexpr int kMaxFft = 1024;
static constexpr int kRowsPerBlock = 2 * kFftWaves;  // real rows per row-pass workgroup
static constexpr int kPerLane = kMaxFft / 64;        // row / column entries per lane

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
__device__ __forceinline__ float2 rot(float2 a, bool inv) {
  return inv ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// Order this wavefront's LDS accesses: writes before the barrier are seen
// by reads after it in every lane of the wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Radix-R DFT of v in registers (forward roots exp(-2 pi i / R); the
// inverse uses their conjugates).
template <int R>
__device__ __forceinline__ void butterfly(float2 (&v)[R], bool inv) {
  if constexpr (R == 2) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 8) {
    // radix 2 x 4: a_n = v_n + v_{n+4} gives the even outputs, b_n =
    // (v_n - v_{n+4}) w8^n the odd ones, each through a 4-point DFT
    const float r2 = 0.70710678118654752440f;
    float2 a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = cadd(v[q], v[q + 4]);
      b[q] = csub(v[q], v[q + 4]);
    }
    // b1 *= w8, b2 *= w8^2 = -/+ i, b3 *= w8^3 (forward w8 = (1 - i)/sqrt2)
    {
      const float2 t = b[1];
      b[1] = inv ? make_float2(r2 * (t.x - t.y), r2 * (t.x + t.y))
                 : make_float2(r2 * (t.x + t.y), r2 * (t.y - t.x));
      b[2] = rot(b[2], inv);
      const float2 u = b[3];
      b[3] = inv ? make_float2(-r2 * (u.x + u.y), r2 * (u.x - u.y))
                 : make_float2(r2 * (u.y - u.x), -r2 * (u.x + u.y));
    }
    float2 e0 = cadd(a[0], a[2]), e1 = csub(a[0], a[2]);
    float2 e2 = cadd(a[1], a[3]), e3 = rot(csub(a[1], a[3]), inv);
    float2 o0 = cadd(b[0], b[2]), o1 = csub(b[0], b[2]);
    float2 o2 = cadd(b[1], b[3]), o3 = rot(csub(b[1], b[3]), inv);
    v[0] = cadd(e0, e2);
    v[4] = csub(e0, e2);
    v[2] = cadd(e1, e3);
    v[6] = csub(e1, e3);
    v[1] = cadd(o0, o2);
    v[5] = csub(o0, o2);
    v[3] = cadd(o1, o3);
    v[7] = csub(o1, o3);
  } else if constexpr (R == 4) {
    float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    float2 b0 = cadd(v[1], v[3]), b1 = rot(csub(v[1], v[3]), inv);
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, b1);
    v[3] = csub(a1, b1);
  } else {  // R == 3
    const float s3 = 0.86602540378443864676f;
    float2 t1 = cadd(v[1], v[2]);
    float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
    float2 d = csub(v[1], v[2]);
    float2 t3 = rot(make_float2(s3 * d.x, s3 * d.y), inv);
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  }
}

// One Stockham stage of radix R (compile-time, so the butterfly lives in
// registers): reads src, writes dst.
template <int R>
__device__ __forceinline__ void fft_stage(const float2* src, float2* dst, int L, int Ns, int lgNs,
                                          const float2* tw, bool inv) {
  const int lane = threadIdx.x & 63;
  const int LR = L / R;
  const int step = L / (Ns * R);  // twiddle-table stride; r k step < L
  for (int j = lane; j < LR; j += 64) {
    const int k = j & (Ns - 1);
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * LR];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      float2 w = tw[r * k * step];
      if (inv) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
    butterfly<R>(v, inv);
    const int idxD = ((j >> lgNs) << lgNs) * R + k;  // (j / Ns) Ns R + k
#pragma unroll
    for (int r = 0; r < R; ++r) dst[idxD + r * Ns] = v[r];
  }
}

// In-LDS complex FFT of length L by one wavefront on buf0 (result in buf0),
// scratch buf1, twiddles tw[j] = exp(-2 pi i j / L) in LDS.  Unnormalised;
// the inverse uses conjugate twiddles.  Stockham autosort stages of radix 8
// while possible, then 4 and 2, and the radix-3 stage (L = 3 * 2^a) last, so
// the stride Ns is a power of two wherever it divides.
static __device__ void wave_fft(float2* buf0, float2* buf1, int L, const float2* tw, bool inv) {
  const int lane = threadIdx.x & 63;
  float2* src = buf0;
  float2* dst = buf1;
  int Ns = 1, lgNs = 0, rem = L;
  while (rem > 1) {
    int R;
    if (rem % 8 == 0) {
      R = 8;
      fft_stage<8>(src, dst, L, Ns, lgNs, tw, inv);
    } else if (rem % 4 == 0) {
      R = 4;
      fft_stage<4>(src, dst, L, Ns, lgNs, tw, inv);
    } else if (rem % 2 == 0) {
      R = 2;
      fft_stage<2>(src, dst, L, Ns, lgNs, tw, inv);
    } else {
      R = 3;
      fft_stage<3>(src, dst, L, Ns, lgNs, tw, inv);
    }
    wave_sync();
    float2* t = src;
    src = dst;
    dst = t;
    Ns *= R;
    lgNs += (R == 8) ? 3 : ((R == 4) ? 2 : 1);  // unused after the radix-3 stage
    rem /= R;
  }
  if (src != buf0) {
    for (int j = lane; j < L; j += 64) buf0[j] = src[j];
    wave_sync();
  }
}

// Register-resident transform for L = 64 R = R^S (R = 8: 512, R = 4: 256):
// lane j starts with x[j + 64 r] in v[r] and ends with X[j + 64 r].  The
// stages are the Stockham radix-R steps of wave_fft (same twiddle-table
// entries, same butterflies, so a 512-point transform gives the same bits),
// but the data stay in registers: every stage reads exactly the pattern
// j + 64 r, so only the scattered write between two stages goes through
// LDS, as separate real and imaginary planes padded by one word in eight
// (conflict-free strides for the writes, near conflict-free reads).  The
// twiddles of stages 1..S-1 are loaded once into registers (RegTw) and
// reused by every transform of the wavefront.
template <int R, int S>
struct RegTw {
  float2 w[S - 1][R - 1];
};
template <int R, int S>
__device__ __forceinline__ void reg_tw_load(RegTw<R, S>& T, const float2* __restrict__ tw) {
  constexpr int L = 64 * R;
  const int j = threadIdx.x & 63;
  int Ns = R;
#pragma unroll
  for (int s = 1; s < S; ++s) {
    const int k = j % Ns, step = L / (Ns * R);
#pragma unroll
    for (int r = 1; r < R; ++r) T.w[s - 1][r - 1] = tw[r * k * step];
    Ns *= R;
  }
}
__device__ __forceinline__ int xpad(int e) { return e + (e >> 3); }
// Exchange-area floats a register transform of length L needs (both planes).
__host__ __device__ constexpr int reg_fft_floats(int L) { return 2 * (L + L / 8); }
template <int R, int S>
__device__ __forceinline__ void reg_fft(float2 (&v)[R], const RegTw<R, S>& T, float* xr, bool inv) {
  static_assert(64 * R == (S == 3 ? R * R * R : R * R * R * R), "L = 64 R must equal R^S");
  constexpr int L = 64 * R;
  float* xi = xr + L + L / 8;
  const int j = threadIdx.x & 63;
  int Ns = 1;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (s > 0) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = T.w[s - 1][r - 1];
        if (inv) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
    }
    butterfly<R>(v, inv);
    if (s + 1 < S) {
      const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = xpad(base + r * Ns);
        xr[e] = v[r].x;
        xi[e] = v[r].y;
      }
      wave_sync();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = xpad(j + 64 * r);
        v[r] = make_float2(xr[e], xi[e]);
      }
      wave_sync();
    }
    Ns *= R;
  }
}

// buf[w][1] also holds two half spectra of I/2 + 1 entries each, hence the
// padding beyond kMaxFft.
struct FftShared {
  static_assert(reg_fft_floats(512) <= 2 * (kMaxFft + 8), "exchange area fits one buffer");
  float2 tw[kMaxFft];
  float2 buf[kFftWaves][2][kMaxFft + 8];
  float red[kFftWaves];
  double dred[kFftWaves];
};

__device__ __forceinline__ void load_twiddles(FftShared& S, const float2* __restrict__ tw, int I) {
  for (int t = threadIdx.x; t < I; t += blockDim.x) S.tw[t] = tw[t];
  __syncthreads();
}

// Forward row transform of one wavefront on its two rows (ra, rb hold
// entries lane + 64 q), in registers; the spectrum lands in a in natural
// order, b is the exchange area.
template <int R, int S>
__device__ __forceinline__ void rows_fwd_reg(const float2* __restrict__ tw, const float* ra,
                                             const float* rb, float2* a, float2* b) {
  const int lane = threadIdx.x & 63;
  RegTw<R, S> T;
  reg_tw_load(T, tw);
  float2 v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = make_float2(ra[r], rb[r]);
  reg_fft<R, S>(v, T, reinterpret_cast<float*>(b), false);
#pragma unroll
  for (int r = 0; r < R; ++r) a[lane + 64 * r] = v[r];
  wave_sync();
}

// Symbol of the cone filter at column frequency kx, row index t (frequency
// ky = t or t - I): |rho|^(1/2) for V^-1 (dir > 0), |rho|^(-1/2) for V, with
// 1/|rho| = I / |k| and the DC term 1/c(0).
__device__ __forceinline__ float cone_symbol(int kx, int t, int I, int dir) {
  const float dc = 3.52549435174692f * (float)I;  // 4 ln(1 + sqrt 2) I
  const int ky = (t <= I / 2) ? t : t - I;
  const float k2 = (float)(kx * kx + ky * ky);
  const float c = (k2 > 0.0f) ? (float)I / sqrtf(k2) : dc;  // 1/|rho|
  return (dir > 0) ? rsqrtf(c) : sqrtf(c);
}

// Inverse row transform of one wavefront in registers: pair(t) gives the
// packed spectrum entry ya + i yb at t, emit(q, t, z) consumes the result at
// t = lane + 64 q; x is the exchange area.
template <int R, int S, class Pair, class Emit>
__device__ __forceinline__ void rows_inv_reg(const float2* __restrict__ tw, Pair pair, Emit emit,
                                             float* x) {
  const int lane = threadIdx.x & 63;
  RegTw<R, S> T;
  reg_tw_load(T, tw);
  float2 v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = pair(lane + 64 * r);
  reg_fft<R, S>(v, T, x, true);
#pragma unroll
  for (int r = 0; r < R; ++r) emit(r, lane + 64 * r, v[r]);
}

}  // namespace dg
