// Internal definitions of the D-GAMP-CT library: plan layout, error
// plumbing and the device helpers several kernels share.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/dgampct.h"

namespace dg {

// ---------------------------------------------------------------- errors

void set_error(const std::string& msg);
dg_status hip_fail(hipError_t e, const char* what);

#define DG_ARG_CHECK(cond, msg)         \
  do {                                  \
    if (!(cond)) {                      \
      ::dg::set_error(msg);             \
      return DG_ERR_ARG;                \
    }                                   \
  } while (0)

#define DG_HIP(call)                                     \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return ::dg::hip_fail(e_, #call); \
  } while (0)

#define DG_LAUNCH_CHECK(what)                                 \
  do {                                                        \
    hipError_t e_ = hipGetLastError();                        \
    if (e_ != hipSuccess) return ::dg::hip_fail(e_, what);    \
  } while (0)

// ---------------------------------------------------------------- plan

// One ray as seen by the chord-weight formula: the ray crosses the grid
// along its major axis (columns when |sin theta| >= |cos theta|, "flat";
// rows otherwise, "steep"); at major index k its cross coordinate (row for
// flat rays, column for steep rays, pixel units, pixel centres at integers)
// is q(k) = q0 + m k.  The line position is kept in 32.32 fixed point
// (q0_fx, m_fx), so q(k) is exact integer arithmetic and the pixel index and
// fractional offset it yields are identical wherever they are evaluated;
// FP32 rounding of a coordinate of size I would otherwise shift the line by
// up to I * 2^-24 pixels.  |pl| is the chord through one full pixel step
// (h / max(|cos|, |sin|), mm); pl < 0 marks a steep ray.  m, inv_r = 1/|m|
// (+inf when the ray is axis-aligned) and q0 as floats serve the weight
// formula and the range search.
struct RayLine {
  int64_t q0_fx, m_fx;
  float pl, m, inv_r, q0;
};

// Fan beam, per ray, for the back-projector: the ray's cross coordinate at
// major index k is q(k) = q0 + m k (pixel-index units, as RayLine), with
// q0 = c1 + c2 and m = m1 + m2 split into multiples of a per-ray grain 2^-e
// (c1, m1) and FP32 remainders below half a grain (c2, m2), e chosen so that
// (c1 - p) + m1 k is exact in FP32 for every pixel index p and k of the
// image; q(k) - p is then rounded once, at a magnitude of order one for the
// pixels the ray meets.  The chord fraction is clamp((hw - |q(k) - p|) inv_r
// + off): hw, inv_r as RayLine's (off = 0); an axis-aligned ray has hw = 1/2,
// inv_r = 2^64 and off = 1/2, which gives its step rule (1 inside, 1/2 on
// the edge, 0 outside) in the same expression.  pl: RayLine's pl (its sign
// marks a steep ray).
struct FanRay {
  float c1, m1, c2, m2;
  float hw, inv_r, off, pl;
};
static_assert(sizeof(FanRay) == 32, "two 16-byte loads per ray");

// Per-view data for the pixel-driven back-projector's candidate search.
//  parallel: bin coordinate of a pixel centre (x, y) [px] is
//            u = a*x + b*y + c; candidates are within +-hw of u.
//  fan:      a, b = source position (px); c = central bin; hw = margin in
//            bins added to the per-pixel footprint bound; pad = 1.001 / dgamma.
struct ViewInfo {
  float a, b, c, hw;
  float cx, cy, inv_dg, pad;  // fan: unit vector towards iso, 1/dgamma [1/rad]
};
// Parallel beam, per view, for the back-projector: the pixel in row i,
// column j has the continuous bin coordinate u = P j + Q i + R, and lies
// |u - b| dqa pixels from ray b's line along the ray's cross axis (dqa: the
// cross-coordinate step between neighbouring bins).  Each of P, Q, R is split
// into a multiple of the grain 2^-e (p1, q1, r1) and an FP32 remainder below
// half a grain (p2, q2, r2), e chosen per view so that every partial sum of
// q1 i + p1 j + r1 - b the kernel forms is a multiple of the grain below 2^23
// grains: those sums are exact in FP32, and u - b = (q1 i + p1 j + r1 - b) +
// (q2 i + p2 j + r2) has one rounding of a number of order one.  The chord
// terms are those of the view's rays (RayLine).
struct ViewRay {
  float p1, q1, r1;       // grain parts of P, Q, R
  float p2, q2, r2;       // remainders
  float hwb;              // footprint half-width in bins, with a 1/64-bin margin
  float dqa;
  float hw, inv_r, apl;   // 0.5 + 0.5 |m|, 1/|m|, |pl|
  float hw_ax;            // half a pixel in bins (the step rule of axis-aligned views)
  int32_t flags;          // bit 0: m == 0; bit 1: hwb >= 1 (footprints over more than 2 bins)
  int32_t pad[3];
};
static_assert(sizeof(ViewRay) == 64, "one scalar load per view");

}  // namespace dg

struct dg_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

struct dg_plan {
  dg_geom g;
  int device;
  int32_t I, nv, nb;
  int64_t N, M;
  dg::RayLine* rays;     // device, M
  dg::ViewInfo* views;   // device, nv
  dg::ViewRay* vrays;    // device, nv (parallel beam only, else null)
  dg::FanRay* frays;     // device, M (fan beam only, else null)
  float2* twiddle;       // device, I: exp(-2 pi i t / I)
  int fft_ok;            // I supported by the FFT kernels
  double half_diag_px;   // sqrt(2)/2 (fan candidate search)
  int proj_variant;      // index into kProjSegVariants (autotuned; default 1)
  int nlm_variant;       // non-local means: 0 = 8 wavefronts per tile, 1 = 4 (default 0)
  float* bm3d_tab;       // device, 72: the orthonormal 8-point DCT-II matrix D[u][k]
                         // (FP64 cosines rounded to FP32) then the 8-point Kaiser window
};

namespace dg {

// ---------------------------------------------------------------- devices

// Chord of a ray through one pixel, given the pixel's cross-axis offset
// delta = |q(k) - p| (pixel units): the projection of the pixel square onto
// the line normal is a trapezoid, so the chord is |pl| times the fraction
// clamp((0.5 (1 + r) - delta) / r, 0, 1) with r = |m|; for an axis-aligned
// ray (r = 0) it is a step with value 1/2 on a pixel edge.  The projector and
// back-projector evaluate this one function on identical operands, so A and
// A^T use bit-identical weights.
__device__ __forceinline__ float chord_fraction(float delta, float m, float inv_r) {
  if (m == 0.0f) return delta < 0.5f ? 1.0f : (delta == 0.5f ? 0.5f : 0.0f);
  float hw = __fmaf_rn(0.5f, fabsf(m), 0.5f);
  return fminf(fmaxf(__fmul_rn(hw - delta, inv_r), 0.0f), 1.0f);
}

// Split the fixed-point cross coordinate into floor(q) and q - floor(q).
__device__ __forceinline__ void split_fx(int64_t q, int* p0, float* f) {
  *p0 = (int)(q >> 32);
  *f = (float)(uint32_t)(q & 0xffffffffll) * 2.3283064365386962890625e-10f;  // 2^-32
}

// SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Rademacher probe value b_i in {-1, +1}.
__device__ __forceinline__ float probe_sign(uint64_t seed, int32_t iter, uint64_t i) {
  uint64_t key = seed ^ ((uint64_t)(uint32_t)iter << 32);
  return (splitmix64(key ^ i) & 1ull) ? -1.0f : 1.0f;
}

// Wavefront-level sums (64 lanes).
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_down(v, o, 64));
  return v;
}

// Block sum of one double per thread; result valid in thread 0.
// `sh` must hold blockDim.x / 64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  }
  __syncthreads();
  return t;
}

__device__ __forceinline__ float block_max(float v, float* sh) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  float t = 0.0f;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = fmaxf(t, sh[w]);
  }
  __syncthreads();
  return t;
}

// Deterministic sum of n per-block partials by one block (strided per-thread
// sums in a fixed order, then the block tree); result valid in thread 0.
__device__ __forceinline__ double finish_sum(const double* partials, int n, double* sh) {
  double v = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) v += partials[k];
  return block_sum(v, sh);
}

__device__ __forceinline__ float finish_max(const float* partials, int n, float* sh) {
  float v = 0.0f;
  for (int k = threadIdx.x; k < n; k += blockDim.x) v = fmaxf(v, partials[k]);
  return block_max(v, sh);
}

// Cross-block results are finished by a separate one-block kernel launched
// right after the producer: the kernel boundary makes every block's partial
// visible, which a device-wide fence inside the producer would do only at
// the cost of writing back the L2 of every XCD for every block.

// Batched launches: one grid covers many slices.  prefix[s] is the first
// block of slice s (prefix[0] = 0, prefix[n] = total blocks); a block finds its
// slice by binary search (uniform per block, so it runs on scalar registers).
// The chip's 8 XCDs (each with its own L2) receive a launch's workgroups
// round-robin: workgroup b runs on XCD b % 8.  xcd_block maps the hardware
// index to a logical one under which every XCD's workgroups form one
// contiguous range (XCD x takes logical blocks [x q + min(x, r), ...) with
// q = nblk / 8, r = nblk % 8), so that neighbouring logical blocks, which
// read the same data, share an L2.  A bijection on [0, nblk).
__device__ __forceinline__ int xcd_block(int b, int nblk) {
  const int q = nblk >> 3, r = nblk & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

__device__ __forceinline__ int slice_of(const int* __restrict__ prefix, int n, int b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

// Fourth word of a raw buffer resource on this architecture (no format
// conversion; out-of-range offsets read 0 and drop writes).
static constexpr int kBufferWord3 = 0x00020000;

// Host-side helpers.
inline unsigned int grid_for(int64_t n, int block, int64_t cap = 65535) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned int)g;
}

// Projector / back-projector argument blocks.
struct BpArgs {
  const RayLine* rays;
  const ViewInfo* views;
  const float* sino;
  float* img;
  int I, nv, nb, fan;
  float half_diag;
  const ViewRay* vrays;  // parallel beam: per-view slope terms
  const FanRay* frays;   // fan beam: per-ray lines for the back-projector
};
// Output channel argument block (per slice).  Standalone: zp = p, s_out,
// tau_p_ptr, tau_s_out.  Fused: zp = z, s_io = s (in: s_prev, out: s), scal.
struct ChanArgs {
  int64_t M;
  const float* zp;
  const float* y;
  float* s_io;
  float* s_out;
  const double* tau_p_ptr;
  double* scal;
  double* tau_s_out;
  double i0, fro2, N;
  double* partials;
  int nblk;  // blocks of the launch that writes the partials, for this slice
};

// Projector arguments.  With chan_on the projector also applies the output
// channel to its rays (Alg. 1 step 2, fused form: chan.zp unused, one FP64
// partial of sum(1 - Var/tau_p) per projector workgroup) instead of storing z.
struct ProjArgs {
  const RayLine* rays;
  const float* img;
  const float* img_t;
  float* sino;
  int I;
  int64_t M;
  int chan_on;
  ChanArgs chan;
};
// Per-iteration parameters of a fused output channel.
struct ChanRun {
  int mode;
  int onsager;
  int t;
  double eta_s;
};

struct ChanOut {
  float s;
  float one_minus_v;  // 1 - Var/tau_p
};

// The Poisson output channel for one ray (see channel.hip for the method).
__device__ __forceinline__ ChanOut poisson_channel(float p, float y, float tau_p, float ln_i0,
                                                   int mode) {
  const float ty = tau_p * y;
  const float ln_tp = logf(tau_p);
  const float C = ln_i0 - p;  // F(delta) = delta + ln w - ln tau_p - C
  // starting point: w0 ~ W0(e^xi), xi = ln(tau_p I0) + tau_p y - p
  const float xi = ln_tp + C + ty;
  float w0;
  if (xi > 1.0f) {
    const float lx = logf(xi);
    w0 = xi - lx + lx / xi;
  } else {
    const float e = expf(fmaxf(xi, -80.0f));
    w0 = e / (1.0f + e) * (1.0f + 0.5f * e / (1.0f + e));
  }
  float delta = w0 - ty;
  // Halley on F with F' = (w+1)/w and F'' = -1/w^2, written without 1/w so
  // that no term overflows for small w; Newton when the Halley denominator
  // is not safely positive.
#pragma unroll
  for (int it = 0; it < 5; ++it) {
    const float w = fmaxf(delta + ty, 1e-30f);
    const float F = delta + logf(w) - ln_tp - C;
    const float w1 = w + 1.0f;
    const float den = 2.0f * w1 * w1 + F;
    delta -= (den > w1 * w1) ? 2.0f * F * w1 * w / den : F * w / w1;
  }
  const float w = fmaxf(delta + ty, 1e-30f);
  const float u = 1.0f / (1.0f + w);
  ChanOut o;
  if (mode == DG_CHANNEL_MODE_ONLY) {
    o.s = delta / tau_p;
    o.one_minus_v = 1.0f - u;
    return o;
  }
  const float u2 = u * u;
  o.s = delta / tau_p + 0.5f * w * u2;
  float v = u - 0.5f * w * tau_p * u2 * u + w * w * tau_p * u2 * u2;
  v = fminf(fmaxf(v, 0.0f), 1.0f);
  o.one_minus_v = 1.0f - v;
  return o;
}

// tau_s (and in the iteration: its damping, tau_p, tau_r, status) from the
// output channel's per-block partial sums; one workgroup, result written by
// thread 0.  Lives here so that a later kernel of the iteration can finish
// the channel without a launch of its own.
template <bool kFused>
__device__ void channel_finish_body(const ChanArgs& A, double eta_s, int t, double* red) {
  if (kFused && A.scal[DG_S_STATUS] != 0.0) return;
  const double tot = finish_sum(A.partials, A.nblk, red);
  if (threadIdx.x == 0) {
    const double tau_p = kFused ? A.fro2 * A.scal[DG_S_TAU_X] / (double)A.M : *A.tau_p_ptr;
    double tau_s = tot / ((double)A.M * tau_p);
    if (kFused) {
      double* scal = A.scal;
      if (t > 0) tau_s = eta_s * tau_s + (1.0 - eta_s) * scal[DG_S_TAU_S];
      const double tau_r = A.N / (A.fro2 * tau_s);
      scal[DG_S_TAU_P] = tau_p;
      scal[DG_S_TAU_S] = tau_s;
      scal[DG_S_TAU_R] = tau_r;
      if (!(tau_s > 0.0) || !isfinite(tau_s) || !(tau_r > 0.0) || !isfinite(tau_r))
        scal[DG_S_STATUS] = (double)(t + 1);
    } else {
      *A.tau_s_out = tau_s;
    }
  }
}

// Non-local-means argument block (per slice): image 0 = r, image 1 = r + eps b.
struct NlmArgs {
  const float* r;
  float* out0;
  float* out1;
  int I, S;
  const double* tau_r;
  const double* eps;
  float hfac;
  // optional: finish the Monte-Carlo step here instead of in a separate
  // launch: eps = max(eps_rel * max(eps_part[0..eps_n)), 1e-12), written to
  // *eps_out by the slice's first workgroup (then eps above is unused)
  const float* eps_part;
  int eps_n;
  double eps_rel;
  double* eps_out;
  // optional, inside the iteration (x == nullptr: not fused): the divergence
  // step's per-pixel part in the same launch.  Image 0 workgroups damp x
  // with D(r) and add -b.D(r), image 1 workgroups add b.D(r + eps b), each
  // into its own FP64 partial (div_part[(img g + by) g + bx], g workgroups
  // per side); the scalar finish (DivFinish) runs in the next launch.
  float* x;
  double* scal;
  double* div_part;
};
// Where a denoiser launch may finish the Monte-Carlo step itself.
struct EpsFinish {
  const float* part;
  int n;
  double eps_rel;
  double* out;
};
// Where a non-local-means launch may take over the per-pixel part of the
// divergence step (the separate divergence pass is then skipped): see
// NlmArgs.
struct DivFuse {
  float* x;
  double* scal;
  double* part;  // one FP64 partial per NLM workgroup of the slice
  double eta_x;
  int t;
};
// The divergence step's scalar finish from those partials, done by the first
// row workgroup of the next preconditioner application (part == nullptr:
// nothing pending).
struct DivFinish {
  const double* part;
  int nblk;
  double N;
  const double* eps;
  double* scal;
};

// The scalar part of the divergence step (Alg. 1 step 4): div =
// b^T (D(r + eps b) - D(r)) / (N eps) from the total, then the damped tau_x
// and the status word (t + 1 on a non-finite or non-positive result).
__device__ __forceinline__ void div_update_scalars(double tot, double N, double eps, double* scal,
                                                   double eta_x, int t) {
  const double div = tot / (N * eps);
  const double tau_r = scal[DG_S_TAU_R];
  double tau_x = div > 0.0 ? tau_r * div : 1e-12 * tau_r;
  if (!(div > 0.0)) scal[DG_S_CLAMPS] += 1.0;
  if (t > 0) tau_x = eta_x * tau_x + (1.0 - eta_x) * scal[DG_S_TAU_X];
  scal[DG_S_DIV] = div;
  scal[DG_S_TAU_X] = tau_x;
  if (!isfinite(div) || !(tau_x > 0.0) || !isfinite(tau_x)) scal[DG_S_STATUS] = (double)(t + 1);
}

__device__ __forceinline__ void div_finish_pending(const DivFinish& F, double eta_x, int t,
                                                   double* red) {
  if (F.scal[DG_S_STATUS] != 0.0) return;
  const double tot = finish_sum(F.part, F.nblk, red);
  if (threadIdx.x == 0) div_update_scalars(tot, F.N, *F.eps, F.scal, eta_x, t);
}

// Divergence argument block (per slice).
struct DivArgs {
  int64_t N;
  const float* xden;
  const float* xpert;
  float* x;
  const double* eps;
  double* div_out;
  double* scal;
  double* partials;
  int nblk;
};

// projector variants (march segments per ray) the autotuner chooses from
static constexpr int kProjSegVariants[4] = {2, 4, 8, 16};
static constexpr int kProjNumVariants = 4;
static constexpr int kNlmNumVariants = 2;  // non-local means: 8 or 4 wavefronts per tile
static constexpr int kRaysPerBlock = 64;

// Kernels launched by more than one file.
dg_status launch_transpose(const float* in, float* out, int I, hipStream_t s);
dg_status launch_project(const dg_plan* p, const float* img, const float* img_t, float* sino,
                         hipStream_t s);
dg_status launch_backproject(const dg_plan* p, const float* sino, float* img, hipStream_t s);

// Per-launch argument blocks of the preconditioner passes (one per slice in
// batched launches).
struct RowsFwdArgs {
  const float* in;
  float2* spec;
  const float2* tw;
  int I;
  int fin;        // 1: the row pass also finishes the output channel
  ChanArgs chan;  // (tau_s, tau_r from the channel's partial sums)
  DivFinish dv;   // else, with fin_t >= 0: it finishes a pending divergence step
};
struct ColsArgs {
  float2* spec;
  const float2* tw;
  int I, dir;
};
struct RowsInvArgs {
  const float2* spec;
  const float2* tw;
  int I, epilogue;
  float* out;
  float* out_t;
  const float* x;
  const double* scal;
  float* partials;
};
struct EpsArgs {
  const float* partials;
  int n;
  double eps_rel;
  double* eps_out;
};

// Preconditioner passes.  Epilogue of the last (inverse-row) pass:
enum PrecEpilogue { PREC_PLAIN = 0, PREC_UPDATE_R = 1 };
struct PrecArgs {
  const float* in;
  float* out;
  float* out_t;          // optional transposed copy of out
  float2* spec;          // workspace: (I/2+1) x I complex
  int dir;               // +1: V^-1, -1: V
  int epilogue;          // PREC_*
  const float* x;        // PREC_UPDATE_R: out = x + tau_r * filtered
  const double* scal;    // PREC_UPDATE_R: tau_r = scal[DG_S_TAU_R]
  double* scal_out;      // PREC_UPDATE_R: eps written to scal_out[DG_S_EPS]
  double eps_rel;
  int eps_elsewhere;     // PREC_UPDATE_R: leave the eps finish to the denoiser
  int fin;               // 1: finish the output channel in the row pass
  ChanArgs chan;
  DivFinish dv;          // fin == 0, fin_t >= 0: finish a pending divergence step there
  double fin_eta;        // eta_s (channel) or eta_x (divergence)
  int fin_t;             // the iteration being finished
  float* partials;       // PREC_UPDATE_R: per-block max |r| (I/2 floats)
};
dg_status launch_precondition(const dg_plan* p, const PrecArgs& a, hipStream_t s);
// eps = max(eps_rel * max(partials), 1e-12) into *eps_out (one block).
dg_status launch_eps_finish(const float* partials, int n, double eps_rel, double* eps_out,
                            hipStream_t s);
size_t precond_work_bytes(const dg_plan* p);

}  // namespace dg
