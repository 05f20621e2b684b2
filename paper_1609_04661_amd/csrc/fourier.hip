// Fourier-slice Radon operator (Sec. 2.4, eq. Radon_op: A = F_gamma^-1 Omega F)
// and its adjoint, as a non-uniform FFT with Kaiser-Bessel interpolation.
//
// Forward, for the point-mass image model h^2 mu_ij at the pixel centres:
//   1. deapodise: b = mu / (phi^(x) phi^(y)) (phi^ the kernel's transform),
//      rows flipped so that both axes run with increasing coordinate, placed
//      centred (index - I/2 modulo K) in a K x K complex grid, K = 2 I;
//   2. 2D FFT: a row pass, a transpose, a row pass (the spectrum ends up
//      transposed: T[kx][ky]);
//   3. interpolate at every polar sample (rho_m cos theta_k, rho_m sin
//      theta_k) from the (W + 1)^2 grid neighbours with separable
//      Kaiser-Bessel weights (W = 8, beta from Beatty et al. 2005 for
//      oversampling 2), times h^2 and the phase of the centring;
//   4. radial inverse DFT of every view: sino_k(b) = Re (1 / (N d))
//      sum_m P_k(m) exp(2 pi i rho_m s_b).
// The adjoint runs the transposed steps in reverse: the radial forward DFT,
// a gather onto the grid through a precomputed sparse table (every grid
// point lists the polar samples whose kernel covers it, so the sum is
// deterministic, no atomics), the inverse 2D FFT, and the cropped,
// deapodised, flipped real part.
// Interpolation weights, phases and the sparse table are derived in FP64 on
// the host at plan time; the arithmetic on the device is FP32.
#include <cmath>
#include <new>
#include <vector>

#include "dg_internal.h"
#include "fft_wave.h"

struct dg_fourier {
  int I, K, nv, nb, W;
  double h, d;
  int64_t M;
  float2* twK;     // K: exp(-2 pi i j / K)
  float* deapod;   // I: 1 / phi^((j - I/2) / K)
  float2* twN;     // nb: exp(+2 pi i q / nb)
  float2* pm;      // nb: exp(-2 pi i frac (m - floor(nb/2)) / nb), frac = 1/2 for even nb
  int2* pbase;     // M: first grid index (kx, ky) of the sample's kernel support
  float* pw;       // M x 2 x (W + 1): x weights then y weights
  float2* pphase;  // M: h^2 exp(-2 pi i delta (kappa + nu) / K)
  int* cptr;       // K * K + 1: entries of transposed-grid point g = kx * K + ky
  int* cidx;       // sample index of each entry
  float* cw;       // weight of each entry (the same FP32 product the forward uses)
};

namespace dg {

static constexpr int kFW = 8;          // kernel width (grid units)
static constexpr int kFT = kFW + 1;    // taps per axis
static constexpr int kFThreads = 256;

static double bessel_i0(double x) {
  // power series; x <= 20 here, 60 terms converge to FP64 accuracy
  double s = 1.0, t = 1.0, q = 0.25 * x * x;
  for (int k = 1; k < 200; ++k) {
    t *= q / ((double)k * (double)k);
    s += t;
    if (t < 1e-17 * s) break;
  }
  return s;
}

static double kb(double t, double W, double beta) {
  const double x = 1.0 - (2.0 * t / W) * (2.0 * t / W);
  return x > 0.0 ? bessel_i0(beta * std::sqrt(x)) : 0.0;
}

static double kb_hat(double xi, double W, double beta) {
  const double a = beta * beta - (M_PI * W * xi) * (M_PI * W * xi);
  if (std::fabs(a) < 1e-12) return W;
  const double r = std::sqrt(std::fabs(a));
  return a > 0.0 ? W * std::sinh(r) / r : W * std::sin(r) / r;
}

// ---------------------------------------------------------------- kernels

// K x K grid: deapodised, flipped image centred at (K - I/2 .. I/2) modulo K,
// zero elsewhere.  One thread per grid entry.
__global__ void __launch_bounds__(kFThreads)
fo_pad(const float* __restrict__ img, const float* __restrict__ deapod, float2* __restrict__ G, int I,
       int K) {
  const int64_t e = (int64_t)blockIdx.x * kFThreads + threadIdx.x;
  if (e >= (int64_t)K * K) return;
  const int r = (int)(e / K), c = (int)(e % K);
  const int c0 = I / 2;
  // grid row r holds centred index rt = r (r < K/2) or r - K
  const int rt = r < K / 2 ? r : r - K, ct = c < K / 2 ? c : c - K;
  const int ip = rt + c0, j = ct + c0;  // flipped row index i' and column j
  float v = 0.0f;
  if (ip >= 0 && ip < I && j >= 0 && j < I) v = img[(int64_t)(I - 1 - ip) * I + j] * deapod[ip] * deapod[j];
  G[e] = make_float2(v, 0.0f);
}

// One length-K complex FFT per wavefront along every row of a K x K grid.
struct FoShared {
  float2 tw[kMaxFft];
  float2 buf[kFftWaves][2][kMaxFft];
};
__global__ void __launch_bounds__(kFftThreads) fo_rows(float2* __restrict__ G, const float2* __restrict__ tw,
                                                       int K, int inv) {
  __shared__ FoShared S;
  for (int t = threadIdx.x; t < K; t += blockDim.x) S.tw[t] = tw[t];
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * kFftWaves + w;
  if (row >= K) return;  // wavefront-uniform
  float2* g = G + (int64_t)row * K;
  for (int j = lane; j < K; j += 64) S.buf[w][0][j] = g[j];
  wave_sync();
  wave_fft(S.buf[w][0], S.buf[w][1], K, S.tw, inv != 0);
  for (int j = lane; j < K; j += 64) g[j] = S.buf[w][0][j];
}

__global__ void fo_transpose(const float2* __restrict__ in, float2* __restrict__ out, int K) {
  __shared__ float2 tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int i = by + r, j = bx + threadIdx.x;
    if (i < K && j < K) tile[r][threadIdx.x] = in[(int64_t)i * K + j];
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int i = bx + r, j = by + threadIdx.x;
    if (i < K && j < K) out[(int64_t)i * K + j] = tile[threadIdx.x][r];
  }
}

// P[p] = phase_p sum_a sum_b wx[a] wy[b] T[(kx0 + a) mod K][(ky0 + b) mod K].
__global__ void __launch_bounds__(kFThreads)
fo_interp(const float2* __restrict__ T, const int2* __restrict__ base, const float* __restrict__ pw,
          const float2* __restrict__ phase, float2* __restrict__ P, int64_t M, int K) {
  const int64_t p = (int64_t)blockIdx.x * kFThreads + threadIdx.x;
  if (p >= M) return;
  const int2 b0 = base[p];
  const float* w = pw + p * (2 * kFT);
  const int mask = K - 1;
  float2 acc = make_float2(0.0f, 0.0f);
  for (int a = 0; a < kFT; ++a) {
    const float wx = w[a];
    const float2* row = T + (int64_t)((b0.x + a) & mask) * K;
    float2 s = make_float2(0.0f, 0.0f);
#pragma unroll
    for (int b = 0; b < kFT; ++b) {
      const float2 t = row[(b0.y + b) & mask];
      const float wb = w[kFT + b];
      s.x = __fmaf_rn(wb, t.x, s.x);
      s.y = __fmaf_rn(wb, t.y, s.y);
    }
    acc.x = __fmaf_rn(wx, s.x, acc.x);
    acc.y = __fmaf_rn(wx, s.y, acc.y);
  }
  P[p] = cmul(acc, phase[p]);
}

// sino[k][b] = Re (1/(nb d)) sum_m P[k][m] pm[m] twN[(m - cm)(b - cb0) mod nb]:
// one view per blockIdx.y, bins over blockIdx.x * 64 + lane (64 threads).
__global__ void __launch_bounds__(64)
fo_radial_inv(const float2* __restrict__ P, const float2* __restrict__ twN, const float2* __restrict__ pm,
              float* __restrict__ sino, int nb, float scale) {
  const int k = blockIdx.y;
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= nb) return;
  const int cm = nb / 2, cb0 = (nb - 1) / 2;
  const float2* Pk = P + (int64_t)k * nb;
  // index of m = 0: (-cm)(b - cb0) mod nb, then + (b - cb0) per step
  const int step = (((b - cb0) % nb) + nb) % nb;
  int idx = (int)((((int64_t)(-cm) * (b - cb0)) % nb + nb) % nb);
  float re = 0.0f;
  for (int m = 0; m < nb; ++m) {
    const float2 v = cmul(Pk[m], pm[m]);
    const float2 t = twN[idx];
    re = __fmaf_rn(v.x, t.x, re);
    re = __fmaf_rn(-v.y, t.y, re);
    idx += step;
    if (idx >= nb) idx -= nb;
  }
  sino[(int64_t)k * nb + b] = re * scale;
}

// Adjoint of fo_radial_inv (real input): Q[k][m] = (1/(nb d)) conj(pm[m])
// sum_b s[k][b] conj(twN[(m - cm)(b - cb0) mod nb]).
__global__ void __launch_bounds__(64)
fo_radial_fwd(const float* __restrict__ sino, const float2* __restrict__ twN, const float2* __restrict__ pm,
              float2* __restrict__ Q, int nb, float scale) {
  const int k = blockIdx.y;
  const int m = blockIdx.x * 64 + threadIdx.x;
  if (m >= nb) return;
  const int cm = nb / 2, cb0 = (nb - 1) / 2;
  const float* sk = sino + (int64_t)k * nb;
  const int step = (((m - cm) % nb) + nb) % nb;
  int idx = (int)((((int64_t)(m - cm) * (-cb0)) % nb + nb) % nb);
  float re = 0.0f, im = 0.0f;
  for (int b = 0; b < nb; ++b) {
    const float s = sk[b];
    const float2 t = twN[idx];
    re = __fmaf_rn(s, t.x, re);
    im = __fmaf_rn(-s, t.y, im);
    idx += step;
    if (idx >= nb) idx -= nb;
  }
  const float2 c = pm[m];
  const float2 v = cmul(make_float2(re, im), make_float2(c.x, -c.y));
  Q[(int64_t)k * nb + m] = make_float2(v.x * scale, v.y * scale);
}

// Transposed-grid gather: T[g] = sum over the entries of g of w conj(phase_p) Q[p].
__global__ void __launch_bounds__(kFThreads)
fo_spread(const int* __restrict__ cptr, const int* __restrict__ cidx, const float* __restrict__ cw,
          const float2* __restrict__ phase, const float2* __restrict__ Q, float2* __restrict__ T,
          int64_t KK) {
  const int64_t g = (int64_t)blockIdx.x * kFThreads + threadIdx.x;
  if (g >= KK) return;
  float2 acc = make_float2(0.0f, 0.0f);
  for (int e = cptr[g]; e < cptr[g + 1]; ++e) {
    const int p = cidx[e];
    const float2 ph = phase[p];
    const float2 v = cmul(Q[p], make_float2(ph.x, -ph.y));
    acc.x = __fmaf_rn(cw[e], v.x, acc.x);
    acc.y = __fmaf_rn(cw[e], v.y, acc.y);
  }
  T[g] = acc;
}

// img[i][j] = Re G[row of i' = I-1-i][col of j] * deapod[i'] * deapod[j].
__global__ void __launch_bounds__(kFThreads)
fo_crop(const float2* __restrict__ G, const float* __restrict__ deapod, float* __restrict__ img, int I,
        int K) {
  const int64_t e = (int64_t)blockIdx.x * kFThreads + threadIdx.x;
  if (e >= (int64_t)I * I) return;
  const int i = (int)(e / I), j = (int)(e % I);
  const int ip = I - 1 - i, c0 = I / 2;
  const int r = (ip - c0 + K) % K, c = (j - c0 + K) % K;
  img[e] = G[(int64_t)r * K + c].x * deapod[ip] * deapod[j];
}

static size_t fo_work_layout(const dg_fourier* f, void* base, float2** G, float2** T, float2** P) {
  char* c = (char*)base;
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = c ? c + off : nullptr;
    off += (b + 255) & ~(size_t)255;
    return q;
  };
  const size_t kk = (size_t)f->K * f->K * sizeof(float2);
  float2* g = (float2*)take(kk);
  float2* t = (float2*)take(kk);
  float2* p = (float2*)take((size_t)f->M * sizeof(float2));
  if (G) *G = g;
  if (T) *T = t;
  if (P) *P = p;
  return off;
}

template <class T>
static hipError_t upload(T** dst, const std::vector<T>& v) {
  hipError_t e = hipMalloc(dst, sizeof(T) * (v.empty() ? 1 : v.size()));
  if (e != hipSuccess) return e;
  if (v.empty()) return hipSuccess;
  return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

}  // namespace dg

using namespace dg;

extern "C" dg_status dg_fourier_destroy(dg_fourier* f) {
  if (!f) return DG_OK;
  void* ptrs[] = {f->twK, f->deapod, f->twN, f->pm, f->pbase, f->pw, f->pphase, f->cptr, f->cidx, f->cw};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete f;
  return DG_OK;
}

extern "C" dg_status dg_fourier_create(const dg_geom* g, dg_fourier** out) {
  DG_ARG_CHECK(g && out, "dg_fourier_create: null argument");
  DG_ARG_CHECK(g->kind == DG_GEOM_PARALLEL, "dg_fourier_create: parallel-beam geometries only");
  DG_ARG_CHECK(g->n >= 8 && g->n <= 512 && (g->n & (g->n - 1)) == 0,
               "dg_fourier_create: image side must be a power of two in [8, 512]");
  // n_views * n_bins <= 2^22 keeps the adjoint's table (81 entries per
  // sample) within 32-bit indices
  DG_ARG_CHECK(g->n_views >= 1 && g->n_bins >= 2 && (int64_t)g->n_views * g->n_bins <= (1ll << 22),
               "dg_fourier_create: need 1 <= n_views, 2 <= n_bins, n_views * n_bins <= 2^22");
  DG_ARG_CHECK(g->pixel_mm > 0 && std::isfinite(g->pixel_mm) && g->bin_mm > 0 &&
                   std::isfinite(g->bin_mm) && std::isfinite(g->angle0_rad) &&
                   std::isfinite(g->span_rad),
               "dg_fourier_create: bad pitch or angles");
  dg_fourier* f = new (std::nothrow) dg_fourier();
  if (!f) {
    set_error("dg_fourier_create: host allocation failed");
    return DG_ERR_NOMEM;
  }
  const int I = g->n, K = 2 * I, nv = g->n_views, nb = g->n_bins, W = kFW;
  f->I = I;
  f->K = K;
  f->nv = nv;
  f->nb = nb;
  f->W = W;
  f->h = g->pixel_mm;
  f->d = g->bin_mm;
  f->M = (int64_t)nv * nb;
  const double sigma = 2.0;
  const double beta = M_PI * std::sqrt((W / sigma) * (W / sigma) * (sigma - 0.5) * (sigma - 0.5) - 0.8);
  std::vector<float2> twK(K), twN(nb), pm(nb);
  for (int j = 0; j < K; ++j)
    twK[j] = make_float2((float)std::cos(-2.0 * M_PI * j / K), (float)std::sin(-2.0 * M_PI * j / K));
  for (int q = 0; q < nb; ++q)
    twN[q] = make_float2((float)std::cos(2.0 * M_PI * q / nb), (float)std::sin(2.0 * M_PI * q / nb));
  const int cm = nb / 2;
  const double frac = (nb % 2 == 0) ? 0.5 : 0.0;
  for (int m = 0; m < nb; ++m) {
    const double a = -2.0 * M_PI * frac * (m - cm) / nb;
    pm[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  std::vector<float> deapod(I);
  for (int j = 0; j < I; ++j) deapod[j] = (float)(1.0 / kb_hat((double)(j - I / 2) / K, W, beta));
  // polar samples
  const int64_t M = f->M;
  std::vector<int2> pbase(M);
  std::vector<float> pw((size_t)M * 2 * kFT);
  std::vector<float2> pphase(M);
  const double delta = (double)(I / 2) - 0.5 * (I - 1);
  const double h = g->pixel_mm, d = g->bin_mm;
  for (int k = 0; k < nv; ++k) {
    const double th = g->angle0_rad + k * g->span_rad / nv;
    const double ct = std::cos(th), st = std::sin(th);
    for (int m = 0; m < nb; ++m) {
      const int64_t p = (int64_t)k * nb + m;
      const double rho = (double)(m - cm) / (nb * d);
      const double kap = rho * ct * K * h, nu = rho * st * K * h;
      const int nx0 = (int)std::floor(kap - 0.5 * W), ny0 = (int)std::floor(nu - 0.5 * W);
      pbase[p] = make_int2(((nx0 % K) + K) % K, ((ny0 % K) + K) % K);
      for (int a = 0; a < kFT; ++a) {
        pw[(size_t)p * 2 * kFT + a] = (float)kb(kap - (nx0 + a), W, beta);
        pw[(size_t)p * 2 * kFT + kFT + a] = (float)kb(nu - (ny0 + a), W, beta);
      }
      const double ang = -2.0 * M_PI * delta * (kap + nu) / K;
      pphase[p] = make_float2((float)(h * h * std::cos(ang)), (float)(h * h * std::sin(ang)));
    }
  }
  // sparse table of the adjoint: entries grouped by transposed-grid point
  // g = kx * K + ky (counting sort over all (sample, a, b) contributions)
  const int64_t KK = (int64_t)K * K;
  std::vector<int> cnt(KK + 1, 0);
  for (int64_t p = 0; p < M; ++p)
    for (int a = 0; a < kFT; ++a)
      for (int b = 0; b < kFT; ++b) {
        const int kx = (pbase[p].x + a) & (K - 1), ky = (pbase[p].y + b) & (K - 1);
        cnt[(int64_t)kx * K + ky + 1]++;
      }
  for (int64_t e = 0; e < KK; ++e) cnt[e + 1] += cnt[e];
  std::vector<int> cidx(cnt[KK]);
  std::vector<float> cw(cnt[KK]);
  std::vector<int> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t p = 0; p < M; ++p)
    for (int a = 0; a < kFT; ++a)
      for (int b = 0; b < kFT; ++b) {
        const int kx = (pbase[p].x + a) & (K - 1), ky = (pbase[p].y + b) & (K - 1);
        const int e = fill[(int64_t)kx * K + ky]++;
        cidx[e] = (int)p;
        // the forward multiplies wy[b] into the row sum, then wx[a]: the
        // same FP32 factors, multiplied once here
        cw[e] = pw[(size_t)p * 2 * kFT + a] * pw[(size_t)p * 2 * kFT + kFT + b];
      }
  hipError_t e;
  if ((e = upload(&f->twK, twK)) != hipSuccess || (e = upload(&f->deapod, deapod)) != hipSuccess ||
      (e = upload(&f->twN, twN)) != hipSuccess || (e = upload(&f->pm, pm)) != hipSuccess ||
      (e = upload(&f->pbase, pbase)) != hipSuccess || (e = upload(&f->pw, pw)) != hipSuccess ||
      (e = upload(&f->pphase, pphase)) != hipSuccess || (e = upload(&f->cptr, cnt)) != hipSuccess ||
      (e = upload(&f->cidx, cidx)) != hipSuccess || (e = upload(&f->cw, cw)) != hipSuccess) {
    dg_fourier_destroy(f);
    return hip_fail(e, "dg_fourier_create: device tables");
  }
  *out = f;
  return DG_OK;
}

extern "C" size_t dg_fourier_workspace_bytes(const dg_fourier* f) {
  return f ? fo_work_layout(f, nullptr, nullptr, nullptr, nullptr) : 0;
}

static dg_status fo_fft2(const dg_fourier* f, float2* G, float2* T, int inv, hipStream_t st) {
  // rows of G, transpose into T, rows of T
  const unsigned int rb = (unsigned int)((f->K + kFftWaves - 1) / kFftWaves);
  hipLaunchKernelGGL(fo_rows, dim3(rb), dim3(kFftThreads), 0, st, G, f->twK, f->K, inv);
  DG_LAUNCH_CHECK("fo_rows");
  const dim3 tg((f->K + 31) / 32, (f->K + 31) / 32), tb(32, 8);
  hipLaunchKernelGGL(fo_transpose, tg, tb, 0, st, G, T, f->K);
  DG_LAUNCH_CHECK("fo_transpose");
  hipLaunchKernelGGL(fo_rows, dim3(rb), dim3(kFftThreads), 0, st, T, f->twK, f->K, inv);
  DG_LAUNCH_CHECK("fo_rows");
  return DG_OK;
}

extern "C" dg_status ct_project_fourier(const dg_fourier* f, const float* img, float* sino, void* work,
                                        void* stream) {
  DG_ARG_CHECK(f && img && sino && work, "ct_project_fourier: null argument");
  hipStream_t st = (hipStream_t)stream;
  float2 *G, *T, *P;
  fo_work_layout(f, work, &G, &T, &P);
  const int64_t KK = (int64_t)f->K * f->K;
  hipLaunchKernelGGL(fo_pad, dim3((unsigned int)((KK + kFThreads - 1) / kFThreads)), dim3(kFThreads), 0,
                     st, img, f->deapod, G, f->I, f->K);
  DG_LAUNCH_CHECK("fo_pad");
  dg_status rc = fo_fft2(f, G, T, 0, st);
  if (rc != DG_OK) return rc;
  hipLaunchKernelGGL(fo_interp, dim3((unsigned int)((f->M + kFThreads - 1) / kFThreads)), dim3(kFThreads),
                     0, st, T, f->pbase, f->pw, f->pphase, P, f->M, f->K);
  DG_LAUNCH_CHECK("fo_interp");
  hipLaunchKernelGGL(fo_radial_inv, dim3((unsigned int)((f->nb + 63) / 64), (unsigned int)f->nv), dim3(64),
                     0, st, P, f->twN, f->pm, sino, f->nb, (float)(1.0 / (f->nb * f->d)));
  DG_LAUNCH_CHECK("fo_radial_inv");
  return DG_OK;
}

extern "C" dg_status ct_backproject_fourier(const dg_fourier* f, const float* sino, float* img, void* work,
                                            void* stream) {
  DG_ARG_CHECK(f && img && sino && work, "ct_backproject_fourier: null argument");
  hipStream_t st = (hipStream_t)stream;
  float2 *G, *T, *P;
  fo_work_layout(f, work, &G, &T, &P);
  const int64_t KK = (int64_t)f->K * f->K;
  hipLaunchKernelGGL(fo_radial_fwd, dim3((unsigned int)((f->nb + 63) / 64), (unsigned int)f->nv), dim3(64),
                     0, st, sino, f->twN, f->pm, P, f->nb, (float)(1.0 / (f->nb * f->d)));
  DG_LAUNCH_CHECK("fo_radial_fwd");
  hipLaunchKernelGGL(fo_spread, dim3((unsigned int)((KK + kFThreads - 1) / kFThreads)), dim3(kFThreads), 0,
                     st, f->cptr, f->cidx, f->cw, f->pphase, P, T, KK);
  DG_LAUNCH_CHECK("fo_spread");
  // inverse 2D FFT from the transposed layout: rows of T, transpose into G, rows of G
  dg_status rc = fo_fft2(f, T, G, 1, st);
  if (rc != DG_OK) return rc;
  hipLaunchKernelGGL(fo_crop, dim3((unsigned int)(((int64_t)f->I * f->I + kFThreads - 1) / kFThreads)),
                     dim3(kFThreads), 0, st, G, f->deapod, img, f->I, f->K);
  DG_LAUNCH_CHECK("fo_crop");
  return DG_OK;
}
