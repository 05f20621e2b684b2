// Ray-driven projector A and pixel-driven back-projector A^T (Sec. 2.1,
// eq. linCT) with exact chord-length weights from one shared formula.
//
// Projector: ray-driven.  A ray marches along its major axis; at each major
// index k it meets at most two pixels across (cross coordinate
// q(k) = q0 + m k, candidates floor(q) and floor(q) + 1).  Threads of a
// wavefront hold consecutive bins of one view, so for steep rays they read
// consecutive columns of one image row.  Flat rays read the transposed copy
// of the image when one is supplied, which makes their reads consecutive too;
// with it, every step reads its two candidates as one 64-bit word of its row
// and weights each word at its own distance from the line (project_body).
//
// Back-projector: pixel-driven (fan beam: one thread per pixel; parallel
// beam: a lane takes four rows of one column and sixteen lanes share a
// column's views, their sums added in a fixed order).  For every view it
// finds the few bins whose footprint covers the pixel and adds weight * s
// for each, with the projector's chord formula evaluated at the pixel's
// distance to each line: parallel beam from the view's bin-coordinate map,
// fan beam from per-ray line records, both split into exact FP32 grain sums
// plus one rounding (so A and A^T are adjoint to FP32 rounding); no atomics,
// so the result is deterministic.
#include "dg_internal.h"

namespace dg {

// back-projector workgroups: 64 columns x kBpBlockY rows (fan and mixed
// batches); the parallel-only kernel's shape is set below (kBpRows)
static constexpr int kBpBlockX = 64, kBpBlockY = 4;

// Block = kRaysPerBlock rays x SEGS segments: wavefront w marches segment w
// of the union of the major-index ranges of 64 consecutive rays (consecutive
// bins of one view) in lockstep, so each load instruction reads neighbouring
// addresses of one buffer row, and the SEGS partial sums are added in a
// fixed order.  Splitting the march gives SEGS times more
// wavefronts to hide memory latency than one thread per ray.
//
// The march is unrolled by kMarch steps: the offsets and weights of both
// candidates of every step are formed first, so 2 kMarch loads are in flight
// before the first multiply-add.  Out-of-range candidates get an offset past
// the end of the buffer, which a raw buffer load returns as 0.  The accumulation order (k ascending,
// candidate p0 before p0 + 1) and every weight are those of ray_weight, so
// A and A^T stay exact transposes of one another.  Each segment's last
// group of kMarch steps runs whole, with dead loads past its end; 8 steps
// keep enough loads in flight while wasting less there than 16 when a
// variant splits the march into many short segments.
static constexpr int kMarch = 8;

template <int SEGS>
__device__ void project_body(const ProjArgs& A, int blk, float (*part)[kRaysPerBlock],
                             const ChanRun& cr) {
  const int lane = threadIdx.x % kRaysPerBlock, seg = threadIdx.x / kRaysPerBlock;
  const int64_t r = (int64_t)blk * kRaysPerBlock + lane;
  const int I = A.I;
  float acc = 0.0f;
  RayLine L{};
  const bool valid = r < A.M;
  if (valid) L = A.rays[r];
  // Major-index range where q(k) lies in (-1, I): candidates exist only there.
  int k0 = I, k1 = -1;  // a lane without a ray adds nothing to the union below
  if (valid) {
    k0 = 0;
    k1 = I - 1;
    if (L.m != 0.0f) {
      float ka = (-1.0f - L.q0) / L.m, kb = ((float)I - L.q0) / L.m;
      float lo = fmaxf(fminf(ka, kb), -2.0f), hi = fminf(fmaxf(ka, kb), (float)I + 1.0f);
      k0 = max(0, (int)floorf(lo) - 1);
      k1 = min(I - 1, (int)ceilf(hi) + 1);
    } else if (!(L.q0 > -1.0f && L.q0 < (float)I)) {
      k1 = -1;
    }
  }
  // The wavefront marches the union of its 64 rays' ranges in lockstep, so at
  // every step its lanes read one row of the (major-index-row) buffer: the
  // neighbouring rays' candidates are neighbouring addresses (coalesced).  A
  // step outside a ray's own range finds both candidates outside the image
  // (offset past the buffer, reads 0) and adds w * 0 = 0.
  for (int o = 32; o > 0; o >>= 1) {
    k0 = min(k0, __shfl_xor(k0, o, 64));
    k1 = max(k1, __shfl_xor(k1, o, 64));
  }
  if (valid) {
    const bool steep = L.pl < 0.0f;
    // One raw buffer resource (wavefront-uniform) spans the image and, when
    // it lies within 4 GiB of it, the transposed copy.
    const char* pi = (const char*)A.img;
    const char* pt = (const char*)A.img_t;
    const uint64_t nbytes = (uint64_t)I * (uint64_t)I * 4u;
    const char* lo = pi;
    uint64_t span = nbytes;
    unsigned di = 0, dt = 0;
    bool use_t = pt != nullptr;
    if (use_t) {
      const char* lo2 = pi < pt ? pi : pt;
      const uint64_t dist = (uint64_t)((pi < pt ? pt : pi) - lo2);
      if (dist + nbytes <= 0xfffffff0ull) {
        lo = lo2;
        di = (unsigned)(pi - lo2);
        dt = (unsigned)(pt - lo2);
        span = dist + nbytes;
      } else {
        use_t = false;
      }
    }
    // Pixel (row i, col j).  Steep: major = row, cross = col -> img[k*I + p].
    // Flat: major = col, cross = row -> img[p*I + k] = img_t[k*I + p].
    // major_rows: the buffer read is laid out with the major index as its row.
    const bool major_rows = steep || use_t;
    const unsigned boff = (steep || !use_t) ? di : dt;
    const int sk = major_rows ? I : 1, sp = major_rows ? 1 : I;

    // this wavefront's share of [k0, k1]
    const int len = k1 - k0 + 1;
    const int chunk = (len + SEGS - 1) / SEGS;
    const int ka = k0 + seg * chunk;
    const int kb = min(k1, ka + chunk - 1);
    int64_t q = L.q0_fx + L.m_fx * (int64_t)ka;  // exact: advanced by m_fx per step
    // an axis-aligned ray keeps its cross coordinate: constant weights
    const bool axis = (L.m == 0.0f);
    float wc0 = 0.0f, wc1 = 0.0f;
    if (axis) {
      int p0;
      float f;
      split_fx(q, &p0, &f);
      wc0 = chord_fraction(f, L.m, L.inv_r);
      wc1 = chord_fraction(1.0f - f, L.m, L.inv_r);
    }
    const float hw = __fmaf_rn(0.5f, fabsf(L.m), 0.5f);
    // raw buffer loads: 32-bit byte offsets, and an offset past the image
    // (used for candidates outside it) reads 0
    const __amdgpu_buffer_rsrc_t img =
        __builtin_amdgcn_make_buffer_rsrc((void*)lo, (short)0, (int)(unsigned)span, kBufferWord3);
    const unsigned skb = (unsigned)sk * 4u, spb = (unsigned)sp * 4u;
    uint32_t qlo = (uint32_t)(uint64_t)q, qhi = (uint32_t)((uint64_t)q >> 32);
    const uint32_t mlo = (uint32_t)(uint64_t)L.m_fx, mhi = (uint32_t)((uint64_t)L.m_fx >> 32);
    // one step: both candidates' weights (chord_fraction's general branch,
    // written out so that the candidates of all steps of a group are formed
    // before any load is consumed) and the 24-bit offset of the second
    // (full-rate multiplies: kk < I and p0 + 1 lies in [0, I] whenever an
    // offset is used, and both strides are at most 4 I bytes)
    auto step = [&](int kk, int& p0, float& g0, float& g1, unsigned& o1) {
      p0 = (int)qhi;
      const float f = (float)qlo * 2.3283064365386962890625e-10f;  // 2^-32
      const uint32_t nlo = qlo + mlo;
      qhi += mhi + (nlo < qlo ? 1u : 0u);
      qlo = nlo;
      g0 = fminf(fmaxf(__fmul_rn(hw - f, L.inv_r), 0.0f), 1.0f);
      const float d1 = 1.0f - f;
      g1 = fminf(fmaxf(__fmul_rn(hw - d1, L.inv_r), 0.0f), 1.0f);
      if (axis) {
        g0 = wc0;
        g1 = wc1;
      }
      o1 = boff + __umul24((unsigned)kk, skb) + __umul24((unsigned)(p0 + 1), spb);
    };
    if (use_t) {
      // every ray reads a buffer laid out with its major index as the row
      // (spb = 4), so its two candidates are adjacent words: one 64-bit
      // read per step, of words c and c + 1 of row kk with c = p0 clamped
      // to [0, I - 2], which never leaves the row (the word after the last
      // one can lie past the image's allocation).  Each word takes the
      // chord rule at its own distance from the line, f + (p0 - c) and
      // f + (p0 - c - 1): for c = p0 these are the two candidates' f and
      // 1 - f, at the row's ends one word is the in-image candidate (its
      // distance formed exactly) and the other lies a pixel or more from
      // the line (weight 0).  Axis-aligned rays take the same expression
      // with 1/|m| = 2^64 and 1/2 added, which gives their step rule (1
      // inside, 1/2 at distance 1/2, 0 beyond).  A step with no candidate
      // inside reads past the resource (0).
      const float ir = axis ? 0x1p64f : L.inv_r;
      const float oc = axis ? 0.5f : 0.0f;
      const int cmax = I - 2;
      // the march bounds are the same in every lane (a wavefront's union
      // range and its segment): in scalar registers, a step's row offset
      // kk * 4 I is scalar work
      const int kau = __builtin_amdgcn_readfirstlane(ka);
      const int kbu = __builtin_amdgcn_readfirstlane(kb);
      uint64_t qq = (uint64_t)q;
      const uint64_t mq = (uint64_t)L.m_fx;
      for (int k = kau; k <= kbu; k += kMarch) {
        float v[2 * kMarch], w[2 * kMarch];
#pragma unroll
        for (int u = 0; u < kMarch; ++u) {
          const int kk = k + u;
          const int p0 = (int)(uint32_t)(qq >> 32);
          const float f = (float)(uint32_t)qq * 2.3283064365386962890625e-10f;  // 2^-32
          qq += mq;
          // an empty statement that keeps the compiler from replacing this
          // one running sum by a separate 64-bit sum per unrolled step
          asm volatile("" : "+v"(qq));
          const int c = min(max(p0, 0), cmax);
          const float fd = (float)(p0 - c);
          const float xa = f + fd, xb = f + (fd - 1.0f);
          w[2 * u] = fminf(fmaxf(__fmaf_rn(hw - fabsf(xa), ir, oc), 0.0f), 1.0f);
          w[2 * u + 1] = fminf(fmaxf(__fmaf_rn(hw - fabsf(xb), ir, oc), 0.0f), 1.0f);
          const bool ok = kk <= kbu && (unsigned)p0 + 1u <= (unsigned)I;
          const unsigned off = ok ? boff + (unsigned)kk * skb + ((unsigned)c << 2) : 0xfffffff0u;
          const auto w2 = __builtin_amdgcn_raw_buffer_load_b64(img, off, 0, 0);
          v[2 * u] = __int_as_float((int)w2[0]);
          v[2 * u + 1] = __int_as_float((int)w2[1]);
        }
#pragma unroll
        for (int e = 0; e < 2 * kMarch; ++e) acc = __fmaf_rn(w[e], v[e], acc);
      }
    } else {
      for (int k = ka; k <= kb; k += kMarch) {
        float v[2 * kMarch], w[2 * kMarch];
#pragma unroll
        for (int u = 0; u < kMarch; ++u) {
          const int kk = k + u;
          int p0;
          unsigned o1;
          step(kk, p0, w[2 * u], w[2 * u + 1], o1);
          const bool live = kk <= kb;
          const unsigned off0 = (live && (unsigned)p0 < (unsigned)I) ? o1 - spb : 0xffffffffu;
          const unsigned off1 = (live && (unsigned)(p0 + 1) < (unsigned)I) ? o1 : 0xffffffffu;
          v[2 * u] = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(img, off0, 0, 0));
          v[2 * u + 1] = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(img, off1, 0, 0));
        }
#pragma unroll
        for (int e = 0; e < 2 * kMarch; ++e) acc = __fmaf_rn(w[e], v[e], acc);
      }
    }
  }
  part[seg][lane] = acc;
  __syncthreads();
  if (seg != 0) return;
  float z = 0.0f;
  if (r < A.M) {
    z = part[0][lane];
#pragma unroll
    for (int g = 1; g < SEGS; ++g) z += part[g][lane];
    z *= fabsf(L.pl);
    if (!A.chan_on) A.sino[r] = z;
  }
  if (!A.chan_on) return;
  // fused output channel on wavefront 0 (this workgroup's 64 rays): as
  // channel_body, frozen once the status word is set
  const ChanArgs& C = A.chan;
  if (C.scal[DG_S_STATUS] != 0.0) return;
  const double tau_p_d = C.fro2 * C.scal[DG_S_TAU_X] / (double)C.M;
  const float tau_p = (float)tau_p_d;
  double one_minus_v = 0.0;
  if (r < A.M) {
    float p = z;
    const float s_prev = C.s_io[r];
    if (cr.onsager) p = __fmaf_rn(-tau_p, s_prev, p);
    const ChanOut o = poisson_channel(p, C.y[r], tau_p, (float)log(C.i0), cr.mode);
    float sv = o.s;
    if (cr.t > 0) {
      const float eta = (float)cr.eta_s;
      sv = __fmaf_rn(eta, sv, (1.0f - eta) * s_prev);
    }
    C.s_io[r] = sv;
    one_minus_v = (double)o.one_minus_v;
  }
  const double bs = wave_sum(one_minus_v);
  if (lane == 0) C.partials[blk] = bs;
}

// Consecutive blocks hold consecutive rays, i.e. the bins of one view, and
// a view reads either the image (steep rays) or its transpose (flat rays);
// with the XCD-contiguous block order every XCD's L2 holds the rays of a
// contiguous range of views and so mostly one of the two buffers.
template <int SEGS>
__global__ void __launch_bounds__(kRaysPerBlock * SEGS) project_kernel(ProjArgs A, ChanRun cr) {
  __shared__ float part[SEGS][kRaysPerBlock];
  project_body<SEGS>(A, xcd_block((int)blockIdx.x, (int)gridDim.x), part, cr);
}
template <int SEGS>
__global__ void __launch_bounds__(kRaysPerBlock * SEGS)
project_batch(const ProjArgs* __restrict__ T, const int* __restrict__ prefix, int n, ChanRun cr) {
  __shared__ float part[SEGS][kRaysPerBlock];
  const int b = xcd_block((int)blockIdx.x, (int)gridDim.x);
  const int s = slice_of(prefix, n, b);
  project_body<SEGS>(T[s], b - prefix[s], part, cr);
}

// Weight of pixel (i, j) on a ray: the same fixed-point cross coordinate and
// the same fraction formula as the projector, hence the same value.
// Weight of pixel (i, j) on a ray whose cross coordinate at the pixel's
// major index is p0 + f (p0 = floor): p the pixel's cross index.
// AX: 0 decides the axis-aligned case (m == 0) per call, 1 / 2 are for a
// caller that knows m != 0 / m == 0 (a wavefront-uniform branch).
template <int AX = 0>
__device__ __forceinline__ float ray_weight_pf(int p0, float f, int p, float m, float inv_r,
                                               float pl) {
  // distance from the line to the pixel's near edge: f for candidate p0,
  // 1 - f for p0 + 1 (both exactly |(p - p0) - f|); any other pixel gets
  // |(p - p0) - f| >= 1, which both forms of chord_fraction map to 0
  // (|m| <= 1, so hw <= 1).  No branches.
  const float d = fabsf((float)(p - p0) - f);
  const float hw = __fmaf_rn(0.5f, fabsf(m), 0.5f);
  const float g = fminf(fmaxf(__fmul_rn(hw - d, inv_r), 0.0f), 1.0f);
  const float ga = d < 0.5f ? 1.0f : (d == 0.5f ? 0.5f : 0.0f);
  if (AX == 1) return fabsf(pl) * g;
  if (AX == 2) return fabsf(pl) * ga;
  return fabsf(pl) * (m == 0.0f ? ga : g);
}
__device__ __forceinline__ float ray_weight_parts(int64_t q0_fx, int64_t m_fx, float m, float inv_r,
                                                  float pl, int i, int j) {
  const bool steep = pl < 0.0f;
  int p0;
  float f;
  split_fx(q0_fx + m_fx * (int64_t)(steep ? i : j), &p0, &f);
  return ray_weight_pf(p0, f, steep ? j : i, m, inv_r, pl);
}
__device__ __forceinline__ float ray_weight(const RayLine& L, int i, int j) {
  return ray_weight_parts(L.q0_fx, L.m_fx, L.m, L.inv_r, L.pl, i, j);
}

// Fan angle atan(t) of t = cr / along (along > 0): an odd polynomial in t
// on [0, 1], fitted to atan by weighted least squares on Chebyshev nodes
// (Lawson's reweighting towards the minimax fit; largest error 1.7e-6 rad in
// FP32), and atan(t) = pi/2 - atan(1/t) above 1.  Within 2e-6 rad of atan;
// the candidate bins it selects are widened by more than that.
__device__ __forceinline__ float fan_angle(float cr, float along) {
  const float t = cr * __builtin_amdgcn_rcpf(along);
  const float a = fabsf(t);
  const bool inv = a > 1.0f;
  const float r = inv ? __builtin_amdgcn_rcpf(a) : a;
  const float s = r * r;
  float q = -0.01171912718564272f;
  q = __fmaf_rn(q, s, 0.052647341042757034f);
  q = __fmaf_rn(q, s, -0.1164264902472496f);
  q = __fmaf_rn(q, s, 0.19354039430618286f);
  q = __fmaf_rn(q, s, -0.33262282609939575f);
  q = __fmaf_rn(q, s, 0.9999772310256958f);
  const float p = q * r;
  return copysignf(inv ? 1.5707963267948966f - p : p, t);
}

// A fan ray's chord weight at pixel (row i, column j) from its FanRay
// record: the cross coordinate's distance q(k) - p from exact grain sums
// plus one rounding, then the chord fraction and |pl|.
__device__ __forceinline__ float fan_weight(const FanRay& L, float fi, float fj) {
  const bool steep = L.pl < 0.0f;
  const float k = steep ? fi : fj, p = steep ? fj : fi;
  const float d = __fmaf_rn(L.m1, k, L.c1 - p) + __fmaf_rn(L.m2, k, L.c2);
  return fabsf(L.pl) * fminf(fmaxf(__fmaf_rn(L.hw - fabsf(d), L.inv_r, L.off), 0.0f), 1.0f);
}

// bx, by: block coordinates of a pixel block of kBpBlockX columns and
// bp_block_rows(MODE) rows.
// Views are taken kBpViews at a time: the footprint of the pixel in every
// view of the group is found first and the ray records and sinogram values
// of the first kBpBinsFan (fan) or kBpBinsPar (parallel) bins per view are
// requested together (clamped in-bounds index, weight 0 when the bin is
// outside the footprint), then accumulated in the order view, bin; a longer
// footprint finishes in a plain loop.  A parallel-beam pixel's footprint is
// (|cos| + |sin|) pixel widths long, so two bins cover it whenever a bin is
// wider than 1/sqrt(2) pixel.  The fan kernel is bound by its address unit
// (one 32-byte ray record per bin), so a requested bin that falls outside a
// short footprint is pure cost: it requests one bin per view and loops over
// the rest.
static constexpr int kBpViewsPar = 1, kBpViewsFan = 4, kBpBinsFan = 1, kBpBinsPar = 2, kBpSplit = 16;
// The parallel-only kernel: a lane takes kBpRows consecutive rows of one
// column (they share the view's terms, the column part of its bin-coordinate
// map and the wavefront's scalar work per view), a workgroup is 64 columns x
// kBpRows rows x kBpSplit view shares (16 wavefronts), one view per step.
// Measured at 512^2 with 64 views: 1 row per lane 19.1 us, 2 rows 12.4, 4
// rows 11.1-12.1 over splits of 4, 8 and 16; 8 rows leave too few
// workgroups.  16 shares keep 4 workgroups per compute unit at 512^2 and
// spread 384^2 evenly (11.4 us; 14.2 with 8 shares).
static constexpr int kBpRows = 4, kBpBlockYPar = 1;
// image rows per workgroup of the back-projector kernel of a mode
__host__ __device__ constexpr int bp_block_rows(int mode) {
  return mode == 0 ? kBpBlockYPar * kBpRows : kBpBlockY;
}

// MODE 0: parallel beam, 1: fan beam, 2: either (decided per slice).
template <int MODE>
__device__ void backproject_body(const BpArgs& A, int bx, int by,
                                 float (*red)[kBpRows][kBpBlockYPar][kBpBlockX]) {
  const int I = A.I;
  const int j = bx * kBpBlockX + threadIdx.x;
  const int i = by * kBpBlockY + threadIdx.y;
  const bool inside = i < I && j < I;
  const float x = (float)j - 0.5f * (float)(I - 1);
  const float y = 0.5f * (float)(I - 1) - (float)i;
  float acc = 0.0f;
  if (MODE == 0 || (MODE == 2 && !A.fan)) {
    // parallel beam.  A pixel's continuous bin coordinate u comes from the
    // view's map as an exact FP32 grain part u1 plus a small remainder su
    // (u1 = q1 i + (p1 j + r1), su = q2 i + (p2 j + r2)); u1 - b is exact for
    // every candidate bin b, so u - b is rounded once at a magnitude of order
    // one.  Its distance to ray b's line along the cross axis, (u - b) dqa,
    // enters the chord fraction of chord_fraction with the view's terms: the
    // weights are the projector's up to its 2^-32-pixel line positions and
    // FP32 rounding.  Axis-aligned views (m == 0) give weight 1 inside the
    // pixel's half-width, 1/2 on it: that test is made in bins, where a line
    // through a pixel's edge is an exact tie.  The first candidate bin is
    // ceil(u - hwb), taken from u rounded (error below 2^-7 bins while
    // |u| < 2^16, inside hwb's 1/64-bin margin past the footprint, so no bin
    // of nonzero weight is missed): a footprint shorter than 2 bins lies
    // within it and the next (a bin past the footprint gets weight 0 from the
    // chord formula itself); views whose bins are narrower than 1/sqrt(2)
    // pixel finish longer footprints in a loop.  Sinogram rows are read
    // through buffer resources sized to the row, so bins past the detector's
    // end read 0.
    // In the parallel-only kernel a lane takes kBpRows consecutive rows of
    // one column and kBpSplit threads share a pixel, each taking a
    // contiguous share of the views (more wavefronts in flight to hide the
    // gathers); their sums are added in a fixed order.  The runtime-mode
    // kernel takes one row per thread and walks the same shares in turn with
    // the same arithmetic per pixel and view, so both kernels give identical
    // bits.
    constexpr int kBpViews = kBpViewsPar;
    constexpr int R = (MODE == 0) ? kBpRows : 1;
    // a wavefront is one row group of the block (blockDim.x is 64): its rows
    // and z slice are uniform
    const int h = (MODE == 0) ? __builtin_amdgcn_readfirstlane((int)threadIdx.z) : 0;
    const int h_end = (MODE == 0) ? h + 1 : kBpSplit;
    const int i0 = __builtin_amdgcn_readfirstlane(
        MODE == 0 ? (by * kBpBlockYPar + (int)threadIdx.y) * R : by * kBpBlockY + (int)threadIdx.y);
    const bool live_px = j < I && i0 < I;
    const float jf = (float)j;
    float yf[R];
#pragma unroll
    for (int r = 0; r < R; ++r) yf[r] = (float)(i0 + r);
    const unsigned row_bytes = (unsigned)A.nb * 4u;
    static_assert(kBpBinsPar == 2, "the two candidate bins are read as one 64-bit word");
    float acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0f;
    for (int hh = h; hh < h_end && live_px; ++hh) {
      const int kbeg = A.nv * hh / kBpSplit, kend = A.nv * (hh + 1) / kBpSplit;
      float share[R];
#pragma unroll
      for (int r = 0; r < R; ++r) share[r] = 0.0f;
      // sinogram rows advance with the view; a view past the share's end
      // (odd count) reads through an empty resource and is not accumulated
      const float* srow = A.sino + (int64_t)kbeg * A.nb;
      for (int k0 = kbeg; k0 < kend; k0 += kBpViews, srow += kBpViews * A.nb) {
        int bb[kBpViews][R];
        float du[kBpViews][R], su[kBpViews][R];  // u1 - bb (exact), the remainder of u
        float sv[kBpViews][R][kBpBinsPar];
#pragma unroll
        for (int g = 0; g < kBpViews; ++g) {
          const bool live = k0 + g < kend;
          const ViewRay& v = A.vrays[live ? k0 + g : kend - 1];
          const float c1 = __fmaf_rn(v.p1, jf, v.r1);  // exact
          const float c2 = __fmaf_rn(v.p2, jf, v.r2);
          const __amdgpu_buffer_rsrc_t srs = __builtin_amdgcn_make_buffer_rsrc(
              (void*)(srow + g * A.nb), (short)0, (int)(live ? row_bytes : 0u), kBufferWord3);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const float u1 = __fmaf_rn(v.q1, yf[r], c1);  // exact
            su[g][r] = __fmaf_rn(v.q2, yf[r], c2);
            const float bf = fmaxf(ceilf((u1 - v.hwb) + su[g][r]), 0.0f);
            du[g][r] = u1 - bf;  // exact
            bb[g][r] = (int)bf;
            // both candidate bins in one 64-bit read: each dword past the
            // row's end reads 0 on its own
            const auto w2 = __builtin_amdgcn_raw_buffer_load_b64(srs, (unsigned)bb[g][r] * 4u, 0, 0);
            sv[g][r][0] = __int_as_float((int)w2[0]);
            sv[g][r][1] = __int_as_float((int)w2[1]);
          }
        }
#pragma unroll
        for (int g = 0; g < kBpViews; ++g) {
          if (k0 + g >= kend) continue;  // wavefront-uniform tail of the share
          const int k = k0 + g;
          const ViewRay& v = A.vrays[k];
          if (v.flags & 1) {
            // axis-aligned view: the step rule in bins (hw_ax = half a pixel
            // in bins); 2^64 (hw_ax - |x|) + 1/2 clamps to 1, 1/2 or 0
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const float x0 = du[g][r] + su[g][r];
              const float x1 = x0 - 1.0f;
              const float w0 = __builtin_amdgcn_fmed3f(__fmaf_rn(v.hw_ax - fabsf(x0), 0x1p64f, 0.5f), 0.0f, 1.0f);
              const float w1 = __builtin_amdgcn_fmed3f(__fmaf_rn(v.hw_ax - fabsf(x1), 0x1p64f, 0.5f), 0.0f, 1.0f);
              const float t = __fmaf_rn(w1, sv[g][r][1], w0 * sv[g][r][0]);
              share[r] = __fmaf_rn(v.apl, t, share[r]);
            }
          } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
              // signed distances [px] to the lines of the two candidates
              const float e0 = (du[g][r] + su[g][r]) * v.dqa;
              const float e1 = e0 - v.dqa;
              const float w0 = fminf(fmaxf(__fmul_rn(v.hw - fabsf(e0), v.inv_r), 0.0f), 1.0f);
              const float w1 = fminf(fmaxf(__fmul_rn(v.hw - fabsf(e1), v.inv_r), 0.0f), 1.0f);
              // the view's chord fractions times its values, then times |pl|:
              // the projector's order of operations (it scales each ray's sum)
              const float t = __fmaf_rn(w1, sv[g][r][1], w0 * sv[g][r][0]);
              share[r] = __fmaf_rn(v.apl, t, share[r]);
            }
          }
          if (v.flags & 2) {
            const float* srow = A.sino + (int64_t)k * A.nb;
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const float x0 = du[g][r] + su[g][r];
              const int be = min(bb[g][r] + (int)floorf(x0 + v.hwb), A.nb - 1);
              for (int b = bb[g][r] + kBpBinsPar; b <= be; ++b) {
                const float x = x0 - (float)(b - bb[g][r]);
                const float w = (v.flags & 1)
                    ? __builtin_amdgcn_fmed3f(__fmaf_rn(v.hw_ax - fabsf(x), 0x1p64f, 0.5f), 0.0f, 1.0f)
                    : fminf(fmaxf(__fmul_rn(v.hw - fabsf(x * v.dqa), v.inv_r), 0.0f), 1.0f);
                share[r] = __fmaf_rn(v.apl * w, srow[b], share[r]);
              }
            }
          }
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = (hh == 0) ? share[r] : acc[r] + share[r];
    }
    if (MODE == 0) {
      if (h > 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) red[h - 1][r][threadIdx.y][threadIdx.x] = acc[r];
      }
      __syncthreads();
      if (h == 0 && live_px) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float a = acc[r];
#pragma unroll
          for (int e = 0; e < kBpSplit - 1; ++e) a += red[e][r][threadIdx.y][threadIdx.x];
          if (i0 + r < I) A.img[(int64_t)(i0 + r) * I + j] = a;
        }
      }
    } else if (live_px) {
      A.img[(int64_t)i0 * I + j] = acc[0];
    }
    return;
  }
  if (!inside) return;
  if (MODE == 0) return;
  constexpr int kBpViews = kBpViewsFan;
  const float fi = (float)i, fj = (float)j;
  for (int k0 = 0; k0 < A.nv; k0 += kBpViews) {
    int bb[kBpViews], be[kBpViews];
    FanRay L[kBpViews][kBpBinsFan];
    float sv[kBpViews][kBpBinsFan];
#pragma unroll
    for (int g = 0; g < kBpViews; ++g) {
      const int k = k0 + g;
      bb[g] = 0;
      be[g] = -1;
      if (k < A.nv) {
        const ViewInfo v = A.views[k];
        const float dx = x - v.a, dy = y - v.b;
        const float along = __fmaf_rn(v.cx, dx, v.cy * dy);
        const float cr = __fmaf_rn(v.cx, dy, -(v.cy * dx));
        const float u = __fmaf_rn(fan_angle(cr, along), v.inv_dg, v.c);
        // the pixel's angular half-width seen from the source is at most
        // asin(xs), xs = half diagonal / distance, and asin(xs) <=
        // tan(asin(xs)) = xs / sqrt(1 - xs^2)
        const float xs = A.half_diag * __builtin_amdgcn_rsqf(__fmaf_rn(dx, dx, dy * dy));
        const float tn = xs * __builtin_amdgcn_rsqf(fmaxf(__fmaf_rn(-xs, xs, 1.0f), 1e-6f));
        const float hw = __fmaf_rn(tn, v.pad, v.hw);
        bb[g] = max((int)ceilf(u - hw), 0);
        be[g] = min((int)floorf(u + hw), A.nb - 1);
      }
      const int kc = min(k, A.nv - 1);
      const int64_t row = (int64_t)kc * A.nb;
#pragma unroll
      for (int c = 0; c < kBpBinsFan; ++c) {
        const int b = min(max(bb[g] + c, 0), A.nb - 1);
        L[g][c] = A.frays[row + b];
        sv[g][c] = A.sino[row + b];
      }
    }
#pragma unroll
    for (int g = 0; g < kBpViews; ++g) {
#pragma unroll
      for (int c = 0; c < kBpBinsFan; ++c) {
        const float wgt = (bb[g] + c <= be[g]) ? fan_weight(L[g][c], fi, fj) : 0.0f;
        acc = __fmaf_rn(wgt, sv[g][c], acc);
      }
      if (be[g] - bb[g] + 1 > kBpBinsFan) {
        const int64_t row = (int64_t)(k0 + g) * A.nb;
        for (int b = bb[g] + kBpBinsFan; b <= be[g]; ++b)
          acc = __fmaf_rn(fan_weight(A.frays[row + b], fi, fj), A.sino[row + b], acc);
      }
    }
  }
  A.img[(int64_t)i * I + j] = acc;
}

// Threads per back-projector workgroup: the parallel-only kernel runs
// kBpSplit threads per pixel column (blockDim.z).
__host__ __device__ constexpr int bp_threads(int mode) {
  return mode == 0 ? kBpBlockX * kBpBlockYPar * kBpSplit : kBpBlockX * kBpBlockY;
}
template <int MODE>
__global__ void __launch_bounds__(bp_threads(MODE))
    backproject_kernel(BpArgs A) {
  __shared__ float red[kBpSplit - 1][kBpRows][kBpBlockYPar][kBpBlockX];
  backproject_body<MODE>(A, blockIdx.x, blockIdx.y, red);
}
template <int MODE>
__global__ void __launch_bounds__(bp_threads(MODE))
    backproject_batch(const BpArgs* __restrict__ T, const int* __restrict__ prefix, int n) {
  __shared__ float red[kBpSplit - 1][kBpRows][kBpBlockYPar][kBpBlockX];
  const int s = slice_of(prefix, n, blockIdx.x);
  const BpArgs A = T[s];
  const int local = blockIdx.x - prefix[s];
  const int gx = (A.I + kBpBlockX - 1) / kBpBlockX;
  backproject_body<MODE>(A, local % gx, local / gx, red);
}

__global__ void transpose_kernel(const float* __restrict__ in, float* __restrict__ out, int I) {
  __shared__ float tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int r = threadIdx.y; r < 32; r += 8) {
    int i = by + r, j = bx + threadIdx.x;
    if (i < I && j < I) tile[r][threadIdx.x] = in[(int64_t)i * I + j];
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += 8) {
    int i = bx + r, j = by + threadIdx.x;
    if (i < I && j < I) out[(int64_t)i * I + j] = tile[threadIdx.x][r];
  }
}

dg_status launch_transpose(const float* in, float* out, int I, hipStream_t s) {
  dim3 grid((I + 31) / 32, (I + 31) / 32), block(32, 8);
  hipLaunchKernelGGL(transpose_kernel, grid, block, 0, s, in, out, I);
  DG_LAUNCH_CHECK("transpose_kernel");
  return DG_OK;
}

unsigned int project_blocks(int64_t M) { return (unsigned int)((M + kRaysPerBlock - 1) / kRaysPerBlock); }
// mode: as the back-projector kernels' (0 parallel-only, 1 fan, 2 either)
unsigned int backproject_blocks(int I, int mode) {
  const int rows = bp_block_rows(mode);
  return (unsigned int)(((I + kBpBlockX - 1) / kBpBlockX) * ((I + rows - 1) / rows));
}

// cr applies only when A.chan_on (the fused output channel).
dg_status launch_project_run(int variant, const ProjArgs& A, const ChanRun& cr, hipStream_t s) {
  const dim3 grid(project_blocks(A.M));
  switch (variant) {
    case 0:
      hipLaunchKernelGGL(project_kernel<2>, grid, dim3(kRaysPerBlock * 2), 0, s, A, cr);
      break;
    case 2:
      hipLaunchKernelGGL(project_kernel<8>, grid, dim3(kRaysPerBlock * 8), 0, s, A, cr);
      break;
    case 3:
      hipLaunchKernelGGL(project_kernel<16>, grid, dim3(kRaysPerBlock * 16), 0, s, A, cr);
      break;
    default:
      hipLaunchKernelGGL(project_kernel<4>, grid, dim3(kRaysPerBlock * 4), 0, s, A, cr);
      break;
  }
  DG_LAUNCH_CHECK("project_kernel");
  return DG_OK;
}

dg_status launch_project_variant(int variant, const ProjArgs& A, hipStream_t s) {
  return launch_project_run(variant, A, ChanRun{}, s);
}

dg_status launch_project_batch(int variant, const ProjArgs* T, const int* prefix, int n, int total,
                               const ChanRun& cr, hipStream_t s) {
  switch (variant) {
    case 0:
      hipLaunchKernelGGL(project_batch<2>, dim3(total), dim3(kRaysPerBlock * 2), 0, s, T, prefix, n,
                         cr);
      break;
    case 2:
      hipLaunchKernelGGL(project_batch<8>, dim3(total), dim3(kRaysPerBlock * 8), 0, s, T, prefix, n,
                         cr);
      break;
    case 3:
      hipLaunchKernelGGL(project_batch<16>, dim3(total), dim3(kRaysPerBlock * 16), 0, s, T, prefix,
                         n, cr);
      break;
    default:
      hipLaunchKernelGGL(project_batch<4>, dim3(total), dim3(kRaysPerBlock * 4), 0, s, T, prefix, n,
                         cr);
      break;
  }
  DG_LAUNCH_CHECK("project_batch");
  return DG_OK;
}

// mode: 0 every slice parallel beam, 1 every slice fan beam, 2 mixed.
dg_status launch_backproject_batch(const BpArgs* T, const int* prefix, int n, int total, int mode,
                                   hipStream_t s) {
  const dim3 block(kBpBlockX, kBpBlockY);
  if (mode == 0)
    hipLaunchKernelGGL(backproject_batch<0>, dim3(total), dim3(kBpBlockX, kBpBlockYPar, kBpSplit), 0,
                       s, T, prefix, n);
  else if (mode == 1)
    hipLaunchKernelGGL(backproject_batch<1>, dim3(total), block, 0, s, T, prefix, n);
  else
    hipLaunchKernelGGL(backproject_batch<2>, dim3(total), block, 0, s, T, prefix, n);
  DG_LAUNCH_CHECK("backproject_batch");
  return DG_OK;
}

dg_status launch_project(const dg_plan* p, const float* img, const float* img_t, float* sino,
                         hipStream_t s) {
  ProjArgs A{p->rays, img, img_t, sino, p->I, p->M, 0, ChanArgs{}};
  return launch_project_variant(p->proj_variant, A, s);
}

dg_status launch_backproject(const dg_plan* p, const float* sino, float* img, hipStream_t s) {
  const int mode = p->g.kind == DG_GEOM_FAN ? 1 : 0;
  const int rows = bp_block_rows(mode);
  dim3 grid((p->I + kBpBlockX - 1) / kBpBlockX, (p->I + rows - 1) / rows);
  dim3 block(kBpBlockX, kBpBlockY);
  BpArgs A{p->rays, p->views, sino, img, p->I, p->nv, p->nb, p->g.kind == DG_GEOM_FAN ? 1 : 0,
           (float)p->half_diag_px, p->vrays, p->frays};
  if (A.fan)
    hipLaunchKernelGGL(backproject_kernel<1>, grid, block, 0, s, A);
  else
    hipLaunchKernelGGL(backproject_kernel<0>, grid, dim3(kBpBlockX, kBpBlockYPar, kBpSplit), 0, s, A);
  DG_LAUNCH_CHECK("backproject_kernel");
  return DG_OK;
}

}  // namespace dg

using namespace dg;

extern "C" dg_status ct_project(const dg_plan* p, const float* img, const float* img_t,
                                float* sino, void* stream) {
  DG_ARG_CHECK(p && img && sino, "ct_project: null argument");
  return launch_project(p, img, img_t, sino, (hipStream_t)stream);
}

extern "C" dg_status ct_backproject(const dg_plan* p, const float* sino, float* img,
                                    void* stream) {
  DG_ARG_CHECK(p && sino && img, "ct_backproject: null argument");
  DG_ARG_CHECK((const void*)sino != (const void*)img, "ct_backproject: sino and img alias");
  return launch_backproject(p, sino, img, (hipStream_t)stream);
}
