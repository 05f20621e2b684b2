// Cone preconditioner V^-1 / V (Sec. 2.3, eq. PPFT preconditioner and eq.
// Aprecon): a circulant filter on the I x I grid, applied as
//   rows  : real-to-complex row transforms, two rows per complex FFT
//   cols  : for each of the I/2+1 retained column frequencies, FFT down the
//           column, multiply by the real symbol, inverse FFT
//   rows' : complex-to-real inverse row transforms, two rows per FFT, with
//           an optional fused epilogue r = x + tau_r * (filtered image) and
//           the max |r| reduction that sets the Monte-Carlo step.
// Each FFT runs inside one workgroup in LDS as a Stockham autosort
// transform with radix-4, radix-2 and (for I = 3 * 2^k) one radix-3 stage;
// twiddles come from a table computed in FP64 at plan time.
// The symbol is c(k)^(-1/2) = (|k| / I)^(1/2) for V^-1 and its inverse for
// V, with |k| the integer frequency radius and c(0) = 4 ln(1 + sqrt 2) I.
#include <cmath>

#include "dg_internal.h"

namespace dg {

static constexpr int kFftThreads = 256;
static constexpr int kMaxFft = 1024;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
__device__ __forceinline__ float2 rot(float2 a, bool inv) {
  return inv ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// In-LDS complex FFT of length L on buf0 (result in buf0), scratch buf1.
// Unnormalised; inverse uses conjugate twiddles.  All threads of the block
// must call it.
__device__ void lds_fft(float2* buf0, float2* buf1, int L, const float2* __restrict__ tw,
                        bool inv) {
  float2* src = buf0;
  float2* dst = buf1;
  int Ns = 1;
  int rem = L;
  while (rem > 1) {
    int R;
    if (rem % 3 == 0)
      R = 3;
    else if (rem % 4 == 0)
      R = 4;
    else
      R = 2;
    const int LR = L / R;
    const int step = L / (Ns * R);  // twiddle-table stride
    for (int j = threadIdx.x; j < LR; j += blockDim.x) {
      const int k = j % Ns;
      float2 v[4];
      for (int r = 0; r < R; ++r) v[r] = src[j + r * LR];
      for (int r = 1; r < R; ++r) {
        float2 w = tw[(r * k * step) % L];
        if (inv) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
      if (R == 2) {
        float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
      } else if (R == 4) {
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
      const int idxD = (j / Ns) * Ns * R + k;
      for (int r = 0; r < R; ++r) dst[idxD + r * Ns] = v[r];
    }
    __syncthreads();
    float2* t = src;
    src = dst;
    dst = t;
    Ns *= R;
    rem /= R;
  }
  if (src != buf0) {
    for (int j = threadIdx.x; j < L; j += blockDim.x) buf0[j] = src[j];
    __syncthreads();
  }
}

// Forward row pass: rows 2m, 2m+1 packed as one complex row; the two real
// spectra are separated by conjugate symmetry and stored column-major as
// spec[k][row], k = 0..I/2.
__device__ void rows_fwd_body(const RowsFwdArgs& A, int m, float2* a, float2* b) {
  const int I = A.I;
  const float* r0 = A.in + (int64_t)(2 * m) * I;
  const float* r1 = r0 + I;
  for (int t = threadIdx.x; t < I; t += blockDim.x) a[t] = make_float2(r0[t], r1[t]);
  __syncthreads();
  lds_fft(a, b, I, A.tw, false);
  for (int k = threadIdx.x; k <= I / 2; k += blockDim.x) {
    float2 Z = a[k], Zc = a[(I - k) % I];
    Zc.y = -Zc.y;
    float2 Xa = make_float2(0.5f * (Z.x + Zc.x), 0.5f * (Z.y + Zc.y));
    float2 d = make_float2(0.5f * (Z.x - Zc.x), 0.5f * (Z.y - Zc.y));
    float2 Xb = make_float2(d.y, -d.x);  // d / i
    float2* col = A.spec + (int64_t)k * I;
    col[2 * m] = Xa;
    col[2 * m + 1] = Xb;
  }
}

// Column pass with the symbol multiply.
__device__ void cols_body(const ColsArgs& A, int kx, float2* a, float2* b) {
  const int I = A.I;
  float2* col = A.spec + (int64_t)kx * I;
  for (int t = threadIdx.x; t < I; t += blockDim.x) a[t] = col[t];
  __syncthreads();
  lds_fft(a, b, I, A.tw, false);
  const float dc = 3.52549435174692f * (float)I;  // 4 ln(1 + sqrt 2) I
  for (int t = threadIdx.x; t < I; t += blockDim.x) {
    const int ky = (t <= I / 2) ? t : t - I;
    const float k2 = (float)(kx * kx + ky * ky);
    float c = (k2 > 0.0f) ? (float)I / sqrtf(k2) : dc;  // 1/|rho|
    float h = (A.dir > 0) ? rsqrtf(c) : sqrtf(c);
    a[t] = make_float2(a[t].x * h, a[t].y * h);
  }
  __syncthreads();
  lds_fft(a, b, I, A.tw, true);
  for (int t = threadIdx.x; t < I; t += blockDim.x) col[t] = a[t];
}

// Inverse row pass (two real rows per complex FFT) with epilogue.
__device__ void rows_inv_body(const RowsInvArgs& A, int m, float2* a, float2* b, float* red) {
  const int I = A.I;
  for (int t = threadIdx.x; t < I; t += blockDim.x) {
    float2 ya, yb;
    if (t <= I / 2) {
      ya = A.spec[(int64_t)t * I + 2 * m];
      yb = A.spec[(int64_t)t * I + 2 * m + 1];
    } else {
      ya = A.spec[(int64_t)(I - t) * I + 2 * m];
      yb = A.spec[(int64_t)(I - t) * I + 2 * m + 1];
      ya.y = -ya.y;
      yb.y = -yb.y;
    }
    a[t] = make_float2(ya.x - yb.y, ya.y + yb.x);  // ya + i yb
  }
  __syncthreads();
  lds_fft(a, b, I, A.tw, true);
  const float scale = 1.0f / ((float)I * (float)I);
  const bool upd = A.epilogue == PREC_UPDATE_R;
  const float tau_r = upd ? (float)A.scal[DG_S_TAU_R] : 0.0f;
  float amax = 0.0f;
  for (int t = threadIdx.x; t < I; t += blockDim.x) {
    float v0 = a[t].x * scale, v1 = a[t].y * scale;
    const int64_t i0 = (int64_t)(2 * m) * I + t, i1 = i0 + I;
    if (upd) {
      v0 = __fmaf_rn(tau_r, v0, A.x[i0]);
      v1 = __fmaf_rn(tau_r, v1, A.x[i1]);
      amax = fmaxf(amax, fmaxf(fabsf(v0), fabsf(v1)));
    }
    A.out[i0] = v0;
    A.out[i1] = v1;
    if (A.out_t) {
      A.out_t[(int64_t)t * I + 2 * m] = v0;
      A.out_t[(int64_t)t * I + 2 * m + 1] = v1;
    }
  }
  if (upd) {
    float bm = block_max(amax, red);
    if (threadIdx.x == 0) A.partials[m] = bm;
  }
}

__device__ void eps_body(const EpsArgs& A, float* red) {
  const float gm = finish_max(A.partials, A.n, red);
  if (threadIdx.x == 0) {
    const double e = A.eps_rel * (double)gm;
    *A.eps_out = e > 1e-12 ? e : 1e-12;
  }
}

__global__ void __launch_bounds__(kFftThreads) prec_rows_fwd(RowsFwdArgs A) {
  __shared__ float2 a[kMaxFft], b[kMaxFft];
  rows_fwd_body(A, blockIdx.x, a, b);
}
__global__ void __launch_bounds__(kFftThreads)
prec_rows_fwd_batch(const RowsFwdArgs* __restrict__ T, const int* __restrict__ prefix, int n) {
  __shared__ float2 a[kMaxFft], b[kMaxFft];
  const int s = slice_of(prefix, n, blockIdx.x);
  rows_fwd_body(T[s], blockIdx.x - prefix[s], a, b);
}
__global__ void __launch_bounds__(kFftThreads) prec_cols(ColsArgs A) {
  __shared__ float2 a[kMaxFft], b[kMaxFft];
  cols_body(A, blockIdx.x, a, b);
}
__global__ void __launch_bounds__(kFftThreads)
prec_cols_batch(const ColsArgs* __restrict__ T, const int* __restrict__ prefix, int n) {
  __shared__ float2 a[kMaxFft], b[kMaxFft];
  const int s = slice_of(prefix, n, blockIdx.x);
  cols_body(T[s], blockIdx.x - prefix[s], a, b);
}
__global__ void __launch_bounds__(kFftThreads) prec_rows_inv(RowsInvArgs A) {
  __shared__ float2 a[kMaxFft], b[kMaxFft];
  __shared__ float red[kFftThreads / 64];
  rows_inv_body(A, blockIdx.x, a, b, red);
}
__global__ void __launch_bounds__(kFftThreads)
prec_rows_inv_batch(const RowsInvArgs* __restrict__ T, const int* __restrict__ prefix, int n) {
  __shared__ float2 a[kMaxFft], b[kMaxFft];
  __shared__ float red[kFftThreads / 64];
  const int s = slice_of(prefix, n, blockIdx.x);
  rows_inv_body(T[s], blockIdx.x - prefix[s], a, b, red);
}
__global__ void __launch_bounds__(256) eps_finish_kernel(EpsArgs A) {
  __shared__ float red[4];
  eps_body(A, red);
}
__global__ void __launch_bounds__(256) eps_finish_batch(const EpsArgs* __restrict__ T) {
  __shared__ float red[4];
  eps_body(T[blockIdx.x], red);
}

dg_status launch_eps_finish(const float* partials, int n, double eps_rel, double* eps_out,
                            hipStream_t s) {
  EpsArgs A{partials, n, eps_rel, eps_out};
  hipLaunchKernelGGL(eps_finish_kernel, dim3(1), dim3(256), 0, s, A);
  DG_LAUNCH_CHECK("eps_finish_kernel");
  return DG_OK;
}

dg_status launch_prec_batch(int pass, const void* table, const int* prefix, int n, int total,
                            hipStream_t s) {
  switch (pass) {
    case 0:
      hipLaunchKernelGGL(prec_rows_fwd_batch, dim3(total), dim3(kFftThreads), 0, s,
                         (const RowsFwdArgs*)table, prefix, n);
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
  RowsFwdArgs f{a.in, a.spec, p->twiddle, I};
  hipLaunchKernelGGL(prec_rows_fwd, dim3(I / 2), dim3(kFftThreads), 0, s, f);
  DG_LAUNCH_CHECK("prec_rows_fwd");
  ColsArgs c{a.spec, p->twiddle, I, a.dir};
  hipLaunchKernelGGL(prec_cols, dim3(I / 2 + 1), dim3(kFftThreads), 0, s, c);
  DG_LAUNCH_CHECK("prec_cols");
  RowsInvArgs r{a.spec, p->twiddle, I, a.epilogue, a.out, a.out_t, a.x, a.scal, a.partials};
  hipLaunchKernelGGL(prec_rows_inv, dim3(I / 2), dim3(kFftThreads), 0, s, r);
  DG_LAUNCH_CHECK("prec_rows_inv");
  if (a.epilogue == PREC_UPDATE_R)
    return launch_eps_finish(a.partials, I / 2, a.eps_rel, a.scal_out + DG_S_EPS, s);
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
