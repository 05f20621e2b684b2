// Cone preconditioner V^-1 / V (Sec. 2.4, eq. PPFT preconditioner and eq.
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
#include "fft_wave.h"

namespace dg {

// Forward row pass, workgroup blk: real rows kRowsPerBlock blk onwards,
// wavefront w packs rows 2m, 2m+1 (m = kFftWaves blk + w) as one complex
// row.  The two real spectra are separated by conjugate symmetry and stored
// column-major as spec[k][row], k = 0..I/2; the workgroup writes its rows of
// every k as one contiguous run.
// fin_blk: the workgroup that runs the scalar finish; a workgroup past the
// row blocks (blk >= prec_row_blocks(I)) runs only that.
__device__ void rows_fwd_body(const RowsFwdArgs& A, int blk, FftShared& S, int fin_t,
                              double fin_eta, int fin_blk) {
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
  if (blk == fin_blk) {
    if (A.fin)
      channel_finish_body<true>(A.chan, fin_eta, fin_t, S.dred);
    else if (A.dv.part && fin_t >= 0)
      div_finish_pending(A.dv, fin_eta, fin_t, S.dred);
  }
  if (2 * blk * kFftWaves >= I) return;  // the finish-only workgroup
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
  // the spectrum block, one 16-byte store per row pair: rows 2w and 2w + 1
  // are wavefront w's pair (I is even, and every slice's spectrum and row
  // offset keeps the store 16-byte aligned)
  for (int idx = threadIdx.x; idx < half * (kRowsPerBlock / 2); idx += blockDim.x) {
    const int k = idx >> 2, w = idx & 3;
    const int row = blk * kRowsPerBlock + 2 * w;
    if (row < I) {
      const float2 lo = S.buf[w][1][k], hi = S.buf[w][1][half + k];
      *reinterpret_cast<float4*>(A.spec + (int64_t)k * I + row) = make_float4(lo.x, lo.y, hi.x, hi.y);
    }
  }
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
  // one 16-byte load per row pair (rows 2w, 2w + 1 of column k)
  constexpr int kSpecPer = (kMaxFft / 2 + 1) * (kRowsPerBlock / 2) / kFftThreads + 1;
  float4 sv[kSpecPer];
#pragma unroll
  for (int q = 0; q < kSpecPer; ++q) {
    const int idx = threadIdx.x + kFftThreads * q;
    const int k = idx >> 2, w = idx & 3;
    const int row = blk * kRowsPerBlock + 2 * w;
    sv[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (idx < half * (kRowsPerBlock / 2) && row < I)
      sv[q] = *reinterpret_cast<const float4*>(A.spec + (int64_t)k * I + row);
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
    const int k = idx >> 2, w = idx & 3;
    if (idx < half * (kRowsPerBlock / 2)) {
      S.buf[w][1][k] = make_float2(sv[q].x, sv[q].y);
      S.buf[w][1][half + k] = make_float2(sv[q].z, sv[q].w);
    }
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
    // the transposed copy, four rows per 16-byte store: rows 4q .. 4q + 3 of
    // this block are wavefronts 2q and 2q + 1's row pairs.  Every supported
    // side is a multiple of 4, so a group of four rows lies wholly inside the
    // image or wholly past it, and each store is 16-byte aligned.
    static_assert(kRowsPerBlock == 8, "two groups of four rows per block");
    for (int idx = threadIdx.x; idx < I * 2; idx += blockDim.x) {
      const int t = idx >> 1, q = idx & 1;
      const int row = blk * kRowsPerBlock + 4 * q;
      if (row < I) {
        const float2 a = S.buf[2 * q][1][t], b = S.buf[2 * q + 1][1][t];
        *reinterpret_cast<float4*>(A.out_t + (int64_t)t * I + row) =
            make_float4(a.x, a.y, b.x, b.y);
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
  rows_fwd_body(A, blockIdx.x, S, fin_t, fin_eta, (int)gridDim.x - 1);
}
__global__ void __launch_bounds__(kFftThreads)
prec_rows_fwd_batch(const RowsFwdArgs* __restrict__ T, const int* __restrict__ prefix, int n,
                    int fin_t, double fin_eta) {
  __shared__ FftShared S;
  const int s = slice_of(prefix, n, blockIdx.x);
  rows_fwd_body(T[s], blockIdx.x - prefix[s], S, fin_t, fin_eta, 0);
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
  // one workgroup more than the rows need, for the scalar finish, so that it
  // runs beside the transforms instead of in front of one of them
  hipLaunchKernelGGL(prec_rows_fwd, dim3(prec_row_blocks(I) + 1), dim3(kFftThreads), 0, s, f,
                     a.fin_t, a.fin_eta);
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
