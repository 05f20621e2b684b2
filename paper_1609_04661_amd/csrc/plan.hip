// Plan creation: per-ray line tables (32.32 fixed point for the projector;
// FP32 grain parts and remainders for the fan-beam back-projector), per-view
// candidate-search data and FFT twiddles, all derived in FP64 on the host.
// Error plumbing of the C ABI lives here too.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "dg_internal.h"

namespace dg {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

dg_status hip_fail(hipError_t e, const char* what) {
  char buf[512];
  snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
  g_last_error = buf;
  return DG_ERR_HIP;
}

// cos/sin with exact values at multiples of pi/2 (grid-aligned rays then lie
// exactly on pixel edges, where the half-weight edge rule applies).
static void snapped_cos_sin(double th, double* c, double* s) {
  double q = th / (0.5 * M_PI);
  double k = std::nearbyint(q);
  if (std::fabs(q - k) < 1e-12) {
    long kk = ((long)k % 4 + 4) % 4;
    const double cs[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
    *c = cs[kk][0];
    *s = cs[kk][1];
    return;
  }
  *c = std::cos(th);
  *s = std::sin(th);
}

static double fan_dgamma(const dg_geom& g) {
  if (g.dgamma_rad != 0.0) return g.dgamma_rad;
  double R = g.n * g.pixel_mm / std::sqrt(2.0);
  return 2.0 * std::asin(R / g.dso_mm) / g.n_bins;
}

// The line of a ray with direction (c, s) and signed offset off_mm from the
// iso-centre: cross coordinate q0 + m k at major index k (pixel-index units)
// and chord step pl (its sign marks a steep ray).
static void ray_params(double c, double s, double off_mm, const dg_geom& g, double* q0_out,
                       double* m_out, double* pl_out) {
  const double h = g.pixel_mm;
  const double off = off_mm / h;  // pixel units
  const double half = 0.5 * (g.n - 1);
  double m, q0, pl;
  if (std::fabs(s) >= std::fabs(c)) {  // flat: march over columns, cross = row
    m = c / s;
    q0 = half * (1.0 - m) - off / s;
    pl = h / std::fabs(s);
  } else {  // steep: march over rows, cross = column
    m = s / c;
    q0 = off / c + half * (1.0 - m);
    pl = -h / std::fabs(c);
  }
  *q0_out = q0;
  *m_out = m;
  *pl_out = pl;
}

static RayLine make_ray(double c, double s, double off_mm, const dg_geom& g) {
  RayLine L;
  double m, q0, pl;
  ray_params(c, s, off_mm, g, &q0, &m, &pl);
  const double two32 = 4294967296.0;
  L.q0_fx = std::llround(q0 * two32);
  L.m_fx = std::llround(m * two32);
  L.q0 = (float)q0;
  L.m = (float)m;
  L.pl = (float)pl;
  L.inv_r = (L.m == 0.0f) ? INFINITY : (float)(1.0 / std::fabs((double)L.m));
  return L;
}

// The back-projector's record of a fan ray (FanRay): the line split into
// grain parts and FP32 remainders, and the chord terms of its RayLine L.
static FanRay make_fan_ray(double c, double s, double off_mm, const dg_geom& g, const RayLine& L) {
  double m, q0, pl;
  ray_params(c, s, off_mm, g, &q0, &m, &pl);
  // largest |(c1 - p) + m1 k| over the image's pixel indices, with slack
  const double bound = std::fabs(q0) + std::fabs(m) * (g.n - 1) + g.n + 4.0;
  const int ge = std::min(40, (int)std::floor(std::log2(8388608.0 / bound)));
  const double c1 = std::ldexp(std::nearbyint(std::ldexp(q0, ge)), -ge);
  const double m1 = std::ldexp(std::nearbyint(std::ldexp(m, ge)), -ge);
  FanRay F;
  F.c1 = (float)c1;
  F.m1 = (float)m1;
  F.c2 = (float)(q0 - c1);
  F.m2 = (float)(m - m1);
  if (L.m == 0.0f) {
    F.hw = 0.5f;
    F.inv_r = 18446744073709551616.0f;  // 2^64
    F.off = 0.5f;
  } else {
    // the device's own half-width, __fmaf_rn(0.5f, |m|, 0.5f): 0.5 |m| is
    // exact, so one rounding either way
    F.hw = 0.5f * std::fabs(L.m) + 0.5f;
    F.inv_r = L.inv_r;
    F.off = 0.0f;
  }
  F.pl = L.pl;
  return F;
}

static bool fft_size_ok(int I) {
  if (I < 8 || I > 1024) return false;
  int n = I;
  if (n % 3 == 0) n /= 3;
  while (n % 2 == 0) n /= 2;
  return n == 1;
}

size_t precond_work_bytes(const dg_plan* p) {
  return (size_t)(p->I / 2 + 1) * (size_t)p->I * sizeof(float2);
}

}  // namespace dg

using namespace dg;

extern "C" const char* dg_last_error(void) { return g_last_error.c_str(); }

extern "C" dg_status dg_plan_create(const dg_geom* g, dg_plan** out) {
  DG_ARG_CHECK(g != nullptr && out != nullptr, "dg_plan_create: null argument");
  DG_ARG_CHECK(g->kind == DG_GEOM_PARALLEL || g->kind == DG_GEOM_FAN,
               "dg_plan_create: unknown geometry kind");
  DG_ARG_CHECK(g->n >= 8 && g->n <= 4096, "dg_plan_create: image side must be in [8, 4096]");
  DG_ARG_CHECK(g->n_views >= 1 && g->n_bins >= 1 && (int64_t)g->n_views * g->n_bins <= (1ll << 30),
               "dg_plan_create: bad view or bin count");
  DG_ARG_CHECK(g->pixel_mm > 0 && std::isfinite(g->pixel_mm), "dg_plan_create: pixel_mm must be > 0");
  DG_ARG_CHECK(std::isfinite(g->angle0_rad) && std::isfinite(g->span_rad),
               "dg_plan_create: non-finite angles");
  if (g->kind == DG_GEOM_PARALLEL) {
    DG_ARG_CHECK(g->bin_mm > 0 && std::isfinite(g->bin_mm), "dg_plan_create: bin_mm must be > 0");
    // the back-projector picks candidate bins from FP32 bin coordinates,
    // which needs |u| below 2^16 bins over the whole image
    const double span = std::sqrt(2.0) * g->pixel_mm / g->bin_mm;
    DG_ARG_CHECK(span * (1.5 * g->n + 1.0) + 0.5 * g->n_bins + 8.0 < 65536.0,
                 "dg_plan_create: parallel bins too narrow for the image (bin coordinates reach 2^16)");
  } else {
    DG_ARG_CHECK(g->dso_mm > g->n * g->pixel_mm / std::sqrt(2.0),
                 "dg_plan_create: fan source must lie outside the image's circumscribed circle");
    DG_ARG_CHECK(std::isfinite(g->dgamma_rad), "dg_plan_create: non-finite dgamma");
  }

  dg_plan* p = new (std::nothrow) dg_plan();
  if (!p) {
    set_error("dg_plan_create: host allocation failed");
    return DG_ERR_NOMEM;
  }
  p->g = *g;
  p->I = g->n;
  p->nv = g->n_views;
  p->nb = g->n_bins;
  p->N = (int64_t)g->n * g->n;
  p->M = (int64_t)g->n_views * g->n_bins;
  p->fft_ok = fft_size_ok(g->n) ? 1 : 0;
  p->half_diag_px = std::sqrt(2.0) * 0.5;
  p->proj_variant = 1;
  (void)hipGetDevice(&p->device);

  std::vector<RayLine> rays((size_t)p->M);
  std::vector<ViewInfo> views((size_t)p->nv);
  // fan beam: the back-projector's per-ray records
  std::vector<FanRay> fr(g->kind == DG_GEOM_FAN ? (size_t)p->M : 0);
  const double h = g->pixel_mm;
  const double cb = 0.5 * (g->n_bins - 1);
  if (g->kind == DG_GEOM_PARALLEL) {
    for (int k = 0; k < p->nv; ++k) {
      double th = g->angle0_rad + k * g->span_rad / p->nv, c, s;
      snapped_cos_sin(th, &c, &s);
      for (int b = 0; b < p->nb; ++b)
        rays[(size_t)k * p->nb + b] = make_ray(c, s, (b - cb) * g->bin_mm, *g);
      ViewInfo& v = views[k];
      v.a = (float)(c * h / g->bin_mm);
      v.b = (float)(s * h / g->bin_mm);
      v.c = (float)cb;
      v.hw = (float)(0.5 * (std::fabs(c) + std::fabs(s)) * h / g->bin_mm + 1e-3);
      v.cx = v.cy = v.inv_dg = v.pad = 0.0f;
    }
  } else {
    const double dg_ = fan_dgamma(*g);
    for (int k = 0; k < p->nv; ++k) {
      double beta = g->angle0_rad + k * g->span_rad / p->nv;
      for (int b = 0; b < p->nb; ++b) {
        double gam = (b - cb) * dg_, c, s;
        snapped_cos_sin(beta + gam + 0.5 * M_PI, &c, &s);
        const double off_mm = -g->dso_mm * std::sin(gam);
        rays[(size_t)k * p->nb + b] = make_ray(c, s, off_mm, *g);
        fr[(size_t)k * p->nb + b] = make_fan_ray(c, s, off_mm, *g, rays[(size_t)k * p->nb + b]);
      }
      ViewInfo& v = views[k];
      v.a = (float)(g->dso_mm * std::cos(beta) / h);
      v.b = (float)(g->dso_mm * std::sin(beta) / h);
      v.c = (float)cb;
      // the device's fan angle is within 2e-6 rad of atan; its footprint
      // bound is widened by 0.1 % and this many bins
      v.hw = (float)(4e-6 / dg_ + 1e-3);
      v.cx = (float)(-std::cos(beta));
      v.cy = (float)(-std::sin(beta));
      v.inv_dg = (float)(1.0 / dg_);
      v.pad = (float)(1.001 / dg_);
    }
  }
  std::vector<float2> tw((size_t)p->I);
  for (int t = 0; t < p->I; ++t) {
    double a = -2.0 * M_PI * t / p->I;
    tw[t] = make_float2((float)std::cos(a), (float)std::sin(a));
  }

  // block-matching denoiser tables: orthonormal DCT-II of length 8,
  // D[u][k] = a_u cos(pi (2k + 1) u / 16), then the Kaiser window of beta 2,
  // K[n] = I0(beta sqrt(1 - (2n/7 - 1)^2)) / I0(beta)
  std::vector<float> bt(72);
  for (int u = 0; u < 8; ++u)
    for (int k = 0; k < 8; ++k)
      bt[u * 8 + k] = (float)((u == 0 ? std::sqrt(1.0 / 8.0) : std::sqrt(2.0 / 8.0)) *
                              std::cos(M_PI * (2 * k + 1) * u / 16.0));
  auto i0 = [](double x) {
    double sum = 1.0, t = 1.0, q = 0.25 * x * x;
    for (int k = 1; k < 100; ++k) {
      t *= q / ((double)k * k);
      sum += t;
    }
    return sum;
  };
  for (int n = 0; n < 8; ++n) {
    const double a = 2.0 * n / 7.0 - 1.0;
    bt[64 + n] = (float)(i0(2.0 * std::sqrt(1.0 - a * a)) / i0(2.0));
  }

  hipError_t e;
  p->rays = nullptr;
  p->views = nullptr;
  p->twiddle = nullptr;
  p->vrays = nullptr;
  p->frays = nullptr;
  p->bm3d_tab = nullptr;
  // parallel beam: per-view bin-coordinate map and chord terms for the
  // back-projector
  std::vector<ViewRay> vr;
  if (g->kind == DG_GEOM_PARALLEL) {
    vr.resize((size_t)p->nv);
    for (int k = 0; k < p->nv; ++k) {
      double c, s;
      snapped_cos_sin(g->angle0_rad + k * g->span_rad / p->nv, &c, &s);
      const RayLine& L = rays[(size_t)k * p->nb];
      ViewRay& r = vr[k];
      // u = ua x + ub y + cb for the centred coordinates x = j - half,
      // y = half - i, i.e. P j + Q i + R over the pixel's indices
      const double ua = c * h / g->bin_mm, ub = s * h / g->bin_mm;
      const double half = 0.5 * (p->I - 1);
      const double P = ua, Q = -ub, R = cb + (ub - ua) * half;
      // the largest partial sum (and candidate bin) in grains stays below 2^23
      const double bound = (std::fabs(P) + std::fabs(Q)) * (p->I - 1) + std::fabs(R) +
                           0.5 * (std::fabs(c) + std::fabs(s)) * h / g->bin_mm + 4.0;
      const int ge = std::min(40, (int)std::floor(std::log2(8388608.0 / bound)));
      const double P1 = std::ldexp(std::nearbyint(std::ldexp(P, ge)), -ge);
      const double Q1 = std::ldexp(std::nearbyint(std::ldexp(Q, ge)), -ge);
      const double R1 = std::ldexp(std::nearbyint(std::ldexp(R, ge)), -ge);
      r.p1 = (float)P1;
      r.q1 = (float)Q1;
      r.r1 = (float)R1;
      r.p2 = (float)(P - P1);
      r.q2 = (float)(Q - Q1);
      r.r2 = (float)(R - R1);
      // the cross axis is the row for flat rays (|sin| >= |cos|), the column
      // otherwise; one bin moves a ray by bin / h / |sin| (resp. |cos|) there
      r.dqa = (float)((std::fabs(s) >= std::fabs(c)) ? (g->bin_mm / h) / std::fabs(s)
                                                     : (g->bin_mm / h) / std::fabs(c));
      // the device forms the same half-width as __fmaf_rn(0.5f, |m|, 0.5f):
      // 0.5 |m| is exact, so one rounding either way
      r.hw = 0.5f * std::fabs(L.m) + 0.5f;
      r.inv_r = L.inv_r;
      r.apl = std::fabs(L.pl);
      // the candidate bins come from u rounded to FP32 (error below 2^-7
      // bins while |u| < 2^16): a 1/64-bin margin keeps every bin of nonzero
      // weight among them
      r.hwb = (float)(0.5 * (std::fabs(c) + std::fabs(s)) * h / g->bin_mm + 1.0 / 64.0);
      r.hw_ax = (float)(0.5 * h / g->bin_mm);
      r.flags = (L.m == 0.0f ? 1 : 0) | (r.hwb >= 1.0f ? 2 : 0);
      r.pad[0] = r.pad[1] = r.pad[2] = 0;
    }
  }
  if ((e = hipMalloc(&p->rays, sizeof(RayLine) * rays.size())) != hipSuccess ||
      (e = hipMalloc(&p->views, sizeof(ViewInfo) * views.size())) != hipSuccess ||
      (e = hipMalloc(&p->twiddle, sizeof(float2) * tw.size())) != hipSuccess ||
      (e = hipMalloc(&p->bm3d_tab, sizeof(float) * bt.size())) != hipSuccess ||
      (!vr.empty() && (e = hipMalloc(&p->vrays, sizeof(ViewRay) * vr.size())) != hipSuccess) ||
      (!fr.empty() && (e = hipMalloc(&p->frays, sizeof(FanRay) * fr.size())) != hipSuccess)) {
    dg_plan_destroy(p);
    hip_fail(e, "dg_plan_create: hipMalloc");
    return DG_ERR_NOMEM;
  }
  if ((e = hipMemcpy(p->rays, rays.data(), sizeof(RayLine) * rays.size(), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(p->views, views.data(), sizeof(ViewInfo) * views.size(),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->twiddle, tw.data(), sizeof(float2) * tw.size(), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(p->bm3d_tab, bt.data(), sizeof(float) * bt.size(), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (!vr.empty() && (e = hipMemcpy(p->vrays, vr.data(), sizeof(ViewRay) * vr.size(),
                                     hipMemcpyHostToDevice)) != hipSuccess) ||
      (!fr.empty() && (e = hipMemcpy(p->frays, fr.data(), sizeof(FanRay) * fr.size(),
                                     hipMemcpyHostToDevice)) != hipSuccess)) {
    dg_plan_destroy(p);
    return hip_fail(e, "dg_plan_create: hipMemcpy");
  }
  *out = p;
  return DG_OK;
}

extern "C" dg_status dg_plan_destroy(dg_plan* p) {
  if (!p) return DG_OK;
  if (p->rays) (void)hipFree(p->rays);
  if (p->views) (void)hipFree(p->views);
  if (p->bm3d_tab) (void)hipFree(p->bm3d_tab);
  if (p->twiddle) (void)hipFree(p->twiddle);
  if (p->vrays) (void)hipFree(p->vrays);
  if (p->frays) (void)hipFree(p->frays);
  delete p;
  return DG_OK;
}
