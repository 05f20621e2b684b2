// Cone preconditioner V^-1 / V (Sec. 2.3, eq. PPFT preconditioner and eq.
// Aprecon): a circulant filter on the I x I grid, applied as
//   rows  : real-to-complex row transforms, two rows per complex FFT
//   cols  : for each of the I/2+1 retained column frequencies, FFT down the
//           column, multiply by the real symbol, inverse FFT
//   rows' : complex-to-real inverse row transforms, two rows per FFT, with
//           an optional fused epilogue r = x + tau_r * (filtered image) and
//           the max |r| reduction that sets the Monte-Carlo step.
// Each FFT runs inside one wavefront (four per workgroup, no workgroup
// barrier inside a transform) as a Stockham autosort transform.  For
// I = 512 and 256 the data stay in registers (radix 8 / radix 4 stages, one
// LDS exchange between stages, twiddles in registers); other sides run the
// stages through LDS with radix 8, 4, 2 and (for I = 3 * 2^k) one radix-3
// stage, twiddles staged in LDS.  The twiddle table is computed in FP64 at
// plan time.
// The symbol is c(k)^(-1/2) = (|k| / I)^(1/2) for V^-1 and its inverse for
// V, with |k| the integer frequency radius and c(0) = 4 ln(1 + sqrt 2) I.
#include <cmath>

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
__device__ void wave_fft(float2* buf0, float2* buf1, int L, const float2* tw, bool inv) {
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

// Forward row pass, workgroup blk: real rows kRowsPerBlock blk onwards,
// wavefront w packs rows 2m, 2m+1 (m = kFftWaves blk + w) as one complex
// row.  The two real spectra are separated by conjugate symmetry and stored
// column-major as spec[k][row], k = 0..I/2; the workgroup writes its rows of
// every k as one contiguous run.
__device__ void rows_fwd_body(const RowsFwdArgs& A, int blk, FftShared& S, int fin_t,
                              double fin_eta) {
  const int I = A.I, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int half = I / 2 + 1;
  const int m = blk * kFftWaves + w;
  const bool live = 2 * m < I;
  // the two rows go to registers first, so their loads are in flight while
  // the twiddles are fetched and the channel finish runs
  float ra[kPerLane], rb[kPerLane];
  if (live) {
    const float* r0 = A.in + (int64_t)(2 * m) * I;
    const float* r1 = r0 + I;
#pragma unroll
    for (int q = 0; q < kPerLane; ++q) {
      const int t = lane + 64 * q;
      if (t < I) {
        ra[q] = r0[t];
        rb[q] = r1[t];
      }
    }
  }
  // the output channel's finish (tau_s, tau_r), or a pending divergence
  // step's, saving it a launch of its own
  if (blk == 0) {
    if (A.fin)
      channel_finish_body<true>(A.chan, fin_eta, fin_t, S.dred);
    else if (A.dv.part && fin_t >= 0)
      div_finish_pending(A.dv, fin_eta, fin_t, S.dred);
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
    if (row < I) A.spec[(int64_t)k * I + row] = S.buf[c >> 1][1][(c & 1) * half + k];
  }
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

// Column transform, symbol multiply and inverse transform of one column in
// registers (cv holds entries lane + 64 q), written back in place.
template <int R, int S>
__device__ __forceinline__ void cols_reg(const ColsArgs& A, int kx, const float2* cv, float* x,
                                         float2* col) {
  constexpr int I = 64 * R;
  const int lane = threadIdx.x & 63;
  RegTw<R, S> T;
  reg_tw_load(T, A.tw);
  float2 v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = cv[r];
  reg_fft<R, S>(v, T, x, false);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float h = cone_symbol(kx, lane + 64 * r, I, A.dir);
    v[r] = make_float2(v[r].x * h, v[r].y * h);
  }
  reg_fft<R, S>(v, T, x, true);
#pragma unroll
  for (int r = 0; r < R; ++r) col[lane + 64 * r] = v[r];
}

// Column pass with the symbol multiply: wavefront w of workgroup blk takes
// column frequency kx = kFftWaves blk + w.
__device__ void cols_body(const ColsArgs& A, int blk, FftShared& S) {
  const int I = A.I, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kx = blk * kFftWaves + w;
  const bool live = kx <= I / 2;
  float2* col = A.spec + (int64_t)kx * I;
  // the column's loads are in flight while the twiddles are fetched
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
  if (I == 512 || I == 256) {
    if (!live) return;
    if (I == 512)
      cols_reg<8, 3>(A, kx, cv, reinterpret_cast<float*>(a), col);
    else
      cols_reg<4, 4>(A, kx, cv, reinterpret_cast<float*>(a), col);
    return;
  }
  load_twiddles(S, A.tw, I);
  if (!live) return;
#pragma unroll
  for (int q = 0; q < kPerLane; ++q) {
    const int t = lane + 64 * q;
    if (t < I) a[t] = cv[q];
  }
  wave_sync();
  wave_fft(a, b, I, S.tw, false);
  for (int t = lane; t < I; t += 64) {
    const float h = cone_symbol(kx, t, I, A.dir);
    a[t] = make_float2(a[t].x * h, a[t].y * h);
  }
  wave_sync();
  wave_fft(a, b, I, S.tw, true);
  for (int t = lane; t < I; t += 64) col[t] = a[t];
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

// Inverse row pass (two real rows per complex FFT) with epilogue; workgroup
// blk owns real rows kRowsPerBlock blk onwards and reads / writes them
// (including the transposed copy) in contiguous runs.
__device__ void rows_inv_body(const RowsInvArgs& A, int blk, FftShared& S) {
  const int I = A.I, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int half = I / 2 + 1;
  const int m = blk * kFftWaves + w;
  const bool live = 2 * m < I;
  const bool upd = A.epilogue == PREC_UPDATE_R;
  const bool reg = I == 512 || I == 256;
  // every global load of the workgroup (its spectrum block and, for the r
  // update, its rows of x) is issued before the twiddles are staged
  constexpr int kSpecPer = (kMaxFft / 2 + 1) * kRowsPerBlock / kFftThreads + 1;
  float2 sv[kSpecPer];
#pragma unroll
  for (int q = 0; q < kSpecPer; ++q) {
    const int idx = threadIdx.x + kFftThreads * q;
    const int k = idx / kRowsPerBlock, c = idx % kRowsPerBlock;
    const int row = blk * kRowsPerBlock + c;
    sv[q] = make_float2(0.0f, 0.0f);
    if (idx < half * kRowsPerBlock && row < I) sv[q] = A.spec[(int64_t)k * I + row];
  }
  float xa[kPerLane], xb[kPerLane];
  if (upd && live) {
#pragma unroll
    for (int q = 0; q < kPerLane; ++q) {
      const int t = lane + 64 * q;
      if (t < I) {
        xa[q] = A.x[(int64_t)(2 * m) * I + t];
        xb[q] = A.x[(int64_t)(2 * m + 1) * I + t];
      }
    }
  }
  if (!reg) load_twiddles(S, A.tw, I);
#pragma unroll
  for (int q = 0; q < kSpecPer; ++q) {
    const int idx = threadIdx.x + kFftThreads * q;
    const int k = idx / kRowsPerBlock, c = idx % kRowsPerBlock;
    if (idx < half * kRowsPerBlock) S.buf[c >> 1][1][(c & 1) * half + k] = sv[q];
  }
  __syncthreads();
  float2* a = S.buf[w][0];
  float2* b = S.buf[w][1];
  const float scale = 1.0f / ((float)I * (float)I);
  const float tau_r = upd ? (float)A.scal[DG_S_TAU_R] : 0.0f;
  float amax = 0.0f;
  // the two half spectra of this wavefront's rows, packed as ya + i yb
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
  auto emit = [&](int q, int t, float2 z) {
    float v0 = z.x * scale, v1 = z.y * scale;
    const int64_t i0 = (int64_t)(2 * m) * I + t, i1 = i0 + I;
    if (upd) {
      v0 = __fmaf_rn(tau_r, v0, xa[q]);
      v1 = __fmaf_rn(tau_r, v1, xb[q]);
      amax = fmaxf(amax, fmaxf(fabsf(v0), fabsf(v1)));
    }
    A.out[i0] = v0;
    A.out[i1] = v1;
    b[t] = make_float2(v0, v1);  // staged for the transposed copy
  };
  if (live) {
    if (I == 512) {
      rows_inv_reg<8, 3>(A.tw, pair, emit, reinterpret_cast<float*>(a));
    } else if (I == 256) {
      rows_inv_reg<4, 4>(A.tw, pair, emit, reinterpret_cast<float*>(a));
    } else {
      for (int t = lane; t < I; t += 64) a[t] = pair(t);
      wave_sync();
      wave_fft(a, b, I, S.tw, true);
#pragma unroll
      for (int q = 0; q < kPerLane; ++q) {
        const int t = lane + 64 * q;
        if (t < I) emit(q, t, a[t]);
      }
    }
  }
  if (A.out_t) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < I * kRowsPerBlock; idx += blockDim.x) {
      const int t = idx / kRowsPerBlock, c = idx % kRowsPerBlock;
      const int row = blk * kRowsPerBlock + c;
      if (row < I) {
        const float2 v = S.buf[c >> 1][1][t];
        A.out_t[(int64_t)t * I + row] = (c & 1) ? v.y : v.x;
      }
    }
  }
  if (upd) {
    const float wm = wave_max(amax);
    if (lane == 0) S.red[w] = wm;
    __syncthreads();
    if (threadIdx.x == 0) {
      float bm = 0.0f;
      for (int q = 0; q < kFftWaves; ++q) bm = fmaxf(bm, S.red[q]);
      A.partials[blk] = bm;
    }
  }
}

__device__ void eps_body(const EpsArgs& A, float* red) {
  const float gm = finish_max(A.partials, A.n, red);
  if (threadIdx.x == 0) {
    const double e = A.eps_rel * (double)gm;
    *A.eps_out = e > 1e-12 ? e : 1e-12;
  }
}

__global__ void __launch_bounds__(kFftThreads)
prec_rows_fwd(RowsFwdArgs A, int fin_t, double fin_eta) {
  __shared__ FftShared S;
  rows_fwd_body(A, blockIdx.x, S, fin_t, fin_eta);
}
__global__ void __launch_bounds__(kFftThreads)
prec_rows_fwd_batch(const RowsFwdArgs* __restrict__ T, const int* __restrict__ prefix, int n,
                    int fin_t, double fin_eta) {
  __shared__ FftShared S;
  const int s = slice_of(prefix, n, blockIdx.x);
  rows_fwd_body(T[s], blockIdx.x - prefix[s], S, fin_t, fin_eta);
}
__global__ void __launch_bounds__(kFftThreads) prec_cols(ColsArgs A) {
  __shared__ FftShared S;
  cols_body(A, blockIdx.x, S);
}
__global__ void __launch_bounds__(kFftThreads)
prec_cols_batch(const ColsArgs* __restrict__ T, const int* __restrict__ prefix, int n) {
  __shared__ FftShared S;
  const int s = slice_of(prefix, n, blockIdx.x);
  cols_body(T[s], blockIdx.x - prefix[s], S);
}
__global__ void __launch_bounds__(kFftThreads) prec_rows_inv(RowsInvArgs A) {
  __shared__ FftShared S;
  rows_inv_body(A, blockIdx.x, S);
}
__global__ void __launch_bounds__(kFftThreads)
prec_rows_inv_batch(const RowsInvArgs* __restrict__ T, const int* __restrict__ prefix, int n) {
  __shared__ FftShared S;
  const int s = slice_of(prefix, n, blockIdx.x);
  rows_inv_body(T[s], blockIdx.x - prefix[s], S);
}
__global__ void __launch_bounds__(256) eps_finish_kernel(EpsArgs A) {
  __shared__ float red[4];
  eps_body(A, red);
}
__global__ void __launch_bounds__(256) eps_finish_batch(const EpsArgs* __restrict__ T) {
  __shared__ float red[4];
  eps_body(T[blockIdx.x], red);
}

// Workgroups of the row passes and of the column pass for side I.
int prec_row_blocks(int I) { return (I + kRowsPerBlock - 1) / kRowsPerBlock; }
int prec_col_blocks(int I) { return (I / 2 + 1 + kFftWaves - 1) / kFftWaves; }

dg_status launch_eps_finish(const float* partials, int n, double eps_rel, double* eps_out,
                            hipStream_t s) {
  EpsArgs A{partials, n, eps_rel, eps_out};
  hipLaunchKernelGGL(eps_finish_kernel, dim3(1), dim3(256), 0, s, A);
  DG_LAUNCH_CHECK("eps_finish_kernel");
  return DG_OK;
}

dg_status launch_prec_batch(int pass, const void* table, const int* prefix, int n, int total,
                            int fin_t, double fin_eta, hipStream_t s) {
  switch (pass) {
    case 0:
      hipLaunchKernelGGL(prec_rows_fwd_batch, dim3(total), dim3(kFftThreads), 0, s,
                         (const RowsFwdArgs*)table, prefix, n, fin_t, fin_eta);
      break;
    case 1:
      hipLaunchKernelGGL(prec_cols_batch, dim3(total), dim3(kFftThreads), 0, s,
                         (const ColsArgs*)table, prefix, n);
      break;
    case 2:
      hipLaunchKernelGGL(prec_rows_inv_batch, dim3(total), dim3(kFftThreads), 0, s,
                         (const RowsInvArgs*)table, prefix, n);
      break;
    default:
      hipLaunchKernelGGL(eps_finish_batch, dim3(n), dim3(256), 0, s, (const EpsArgs*)table);
      break;
  }
  DG_LAUNCH_CHECK("prec batch");
  return DG_OK;
}

dg_status launch_precondition(const dg_plan* p, const PrecArgs& a, hipStream_t s) {
  if (!p->fft_ok) {
    set_error("preconditioner: image side must be 2^a or 3*2^a in [8, 1024]");
    return DG_ERR_UNSUPPORTED;
  }
  const int I = p->I;
  RowsFwdArgs f{a.in, a.spec, p->twiddle, I, a.fin, a.chan, a.dv};
  hipLaunchKernelGGL(prec_rows_fwd, dim3(prec_row_blocks(I)), dim3(kFftThreads), 0, s, f, a.fin_t,
                     a.fin_eta);
  DG_LAUNCH_CHECK("prec_rows_fwd");
  ColsArgs c{a.spec, p->twiddle, I, a.dir};
  hipLaunchKernelGGL(prec_cols, dim3(prec_col_blocks(I)), dim3(kFftThreads), 0, s, c);
  DG_LAUNCH_CHECK("prec_cols");
  RowsInvArgs r{a.spec, p->twiddle, I, a.epilogue, a.out, a.out_t, a.x, a.scal, a.partials};
  hipLaunchKernelGGL(prec_rows_inv, dim3(prec_row_blocks(I)), dim3(kFftThreads), 0, s, r);
  DG_LAUNCH_CHECK("prec_rows_inv");
  if (a.epilogue == PREC_UPDATE_R && !a.eps_elsewhere)
    return launch_eps_finish(a.partials, prec_row_blocks(I), a.eps_rel, a.scal_out + DG_S_EPS, s);
  return DG_OK;
}

}  // namespace dg

using namespace dg;

extern "C" dg_status ct_precondition(const dg_plan* p, int32_t dir, const float* in, float* out,
                                     void* work, void* stream) {
  DG_ARG_CHECK(p && in && out && work, "ct_precondition: null argument");
  DG_ARG_CHECK(dir == 1 || dir == -1, "ct_precondition: dir must be +1 (V^-1) or -1 (V)");
  PrecArgs a{};
  a.in = in;
  a.out = out;
  a.out_t = nullptr;
  a.spec = (float2*)work;
  a.dir = dir;
  a.epilogue = PREC_PLAIN;
  return launch_precondition(p, a, (hipStream_t)stream);
}
