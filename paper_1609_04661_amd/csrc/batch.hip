// Many independent slices (uneven image sizes and view counts) run as one
// launch per phase: every batched kernel covers the blocks of all slices, a
// block finds its slice in a per-phase prefix table (see slice_of), and reads
// that slice's argument block.  Small slices that would leave most of the 256
// CUs idle on their own fill the chip together.  The per-slice argument
// tables are built once when buffers are bound; an iteration is then a fixed
// sequence of launches with no host synchronisation, which a HIP graph can
// capture (dg_batch_graph_create).
//
// A small autotuner (dg_batch_autotune / dg_plan_autotune) times the
// projector's march-segmentation variants on the actual geometry and keeps
// the fastest.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "dg_internal.h"

namespace dg {

dg_status launch_prec_batch(int pass, const void* table, const int* prefix, int n, int total,
                            int fin_t, double fin_eta, hipStream_t s);
dg_status launch_project_batch(int variant, const ProjArgs* T, const int* prefix, int n, int total,
                               const ChanRun& cr, hipStream_t s);
dg_status launch_project_variant(int variant, const ProjArgs& A, hipStream_t s);
dg_status launch_backproject_batch(const BpArgs* T, const int* prefix, int n, int total, int mode,
                                   hipStream_t st);
dg_status launch_nlm_batch(int P, int variant, const NlmArgs* T, const int* prefix, int n,
                           int total, uint64_t seed, int iter, double eta_x, int t,
                           hipStream_t st);
dg_status launch_div_finish_batch(const DivArgs* T, int n, double eta_x, int t, hipStream_t st);
dg_status launch_div_batch(const DivArgs* T, const int* prefix, int n, int total, uint64_t seed,
                           int iter, double eta_x, int t, hipStream_t st);
dg_status check_denoise_params(const dg_plan* p, int kind, const void* params);
dg_status cnn_check_params(const dg_plan* p, const void* params);
dg_status cnn_launch_denoise_batch(const void* params, const float* r, const double* scal_eps,
                                   int eps_stride, uint64_t seed, int iter, float* x_den,
                                   float* x_pert, int n, int I, hipStream_t st);
unsigned int project_blocks(int64_t M);
unsigned int backproject_blocks(int I, int mode);
unsigned int red_grid(int64_t N);
unsigned int nlm_blocks(int I);
int prec_row_blocks(int I);
int prec_col_blocks(int I);
dg_status launch_fill(float* p, int64_t n, float v, hipStream_t st);

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
static constexpr int kPartMax = 1024;

__global__ void batch_init_scal(double* scal, int n, double tau_x0) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n * DG_NSCAL) scal[k] = (k % DG_NSCAL == DG_S_TAU_X) ? tau_x0 : 0.0;
}

template <class T>
static dg_status upload(const std::vector<T>& v, T** dev) {
  if (*dev) (void)hipFree(*dev);
  *dev = nullptr;
  if (v.empty()) return DG_OK;
  DG_HIP(hipMalloc(dev, sizeof(T) * v.size()));
  DG_HIP(hipMemcpy(*dev, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return DG_OK;
}

}  // namespace dg

using namespace dg;

struct dg_batch {
  int n = 0;
  std::vector<dg_plan*> plans;
  std::vector<int64_t> img_off, sino_off, spec_off;
  int64_t totN = 0, totM = 0, totSpec = 0;
  int uniform_I = 0;  // side when all slices share it, else 0
  // per-phase block prefixes (host + device)
  std::vector<int> pre_rows, pre_cols, pre_proj, pre_bp, pre_nlm, pre_div;
  int* d_pre_rows = nullptr;
  int* d_pre_cols = nullptr;
  int* d_pre_proj = nullptr;
  int* d_pre_bp = nullptr;
  int* d_pre_nlm = nullptr;
  int* d_pre_div = nullptr;
  // argument tables (device), built by dg_batch_bind
  RowsFwdArgs* t_rf_x = nullptr;
  RowsFwdArgs* t_rf_g = nullptr;
  ColsArgs* t_cols = nullptr;
  RowsInvArgs* t_ri_mu = nullptr;
  RowsInvArgs* t_ri_r = nullptr;
  RowsInvArgs* t_ri_out = nullptr;
  EpsArgs* t_eps = nullptr;
  ProjArgs* t_proj = nullptr;
  ChanArgs* t_chan = nullptr;
  BpArgs* t_bp = nullptr;
  NlmArgs* t_nlm = nullptr;
  DivArgs* t_div = nullptr;
  DivArgs* t_divn = nullptr;  // the NLM-fused divergence's finish
  ProjArgs* t_projc = nullptr;  // the projector with the output channel fused in
  // bound buffers
  bool bound = false;
  float *x = nullptr, *s = nullptr, *mu_out = nullptr;
  double* scal = nullptr;
  const float* y = nullptr;
  float *r = nullptr, *xden = nullptr, *xpert = nullptr;
  int den_kind = DG_DEN_NLM;
  dg_nlm_params nlm{};
  dg_cnn_params cnn{};
  int proj_variant = 1;
  int nlm_variant = 0;
  std::vector<NlmArgs> h_nlm;  // host copy of t_nlm (the tuner times variants on it)
  int bp_mode = 0;  // back-projector kernel: 0 all parallel beam, 1 all fan beam, 2 mixed
};

static size_t batch_work_layout(const dg_batch* b, void* base, char** parts) {
  // parts: spec, mu and mu^T (each slice's pair side by side, so that the
  // projector's buffer resource spans the two at any batch size), unused,
  // z, g, r, xden, xpert, dpart, fpart, npart (NLM
  // divergence partials, per-slice offsets pre_nlm), ppart (the projector's
  // fused-channel partials, offsets pre_proj)
  char* c = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = c ? c + off : nullptr;
    off += a256(bytes);
    return p;
  };
  const size_t nb = sizeof(float) * (size_t)b->totN, mb = sizeof(float) * (size_t)b->totM;
  char* tmp[12];
  tmp[0] = take(sizeof(float2) * (size_t)b->totSpec);
  tmp[1] = take(2 * nb);
  tmp[2] = nullptr;
  tmp[3] = take(mb);
  tmp[4] = take(nb);
  tmp[5] = take(nb);
  tmp[6] = take(nb);
  tmp[7] = take(nb);
  tmp[8] = take(sizeof(double) * (size_t)kPartMax * b->n);
  tmp[9] = take(sizeof(float) * (size_t)kPartMax * b->n);
  tmp[10] = take(sizeof(double) * (size_t)b->pre_nlm[b->n]);
  tmp[11] = take(sizeof(double) * (size_t)b->pre_proj[b->n]);
  if (parts)
    for (int k = 0; k < 12; ++k) parts[k] = tmp[k];
  return off;
}

static void free_tables(dg_batch* b) {
  void* ptrs[] = {b->t_rf_x, b->t_rf_g, b->t_cols, b->t_ri_mu, b->t_ri_r, b->t_ri_out, b->t_eps,
                  b->t_proj, b->t_chan, b->t_bp,  b->t_nlm,  b->t_div, b->t_divn,
                  b->t_projc};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  b->t_rf_x = b->t_rf_g = nullptr;
  b->t_cols = nullptr;
  b->t_ri_mu = b->t_ri_r = b->t_ri_out = nullptr;
  b->t_eps = nullptr;
  b->t_proj = nullptr;
  b->t_chan = nullptr;
  b->t_bp = nullptr;
  b->t_nlm = nullptr;
  b->t_div = nullptr;
  b->t_divn = nullptr;
  b->t_projc = nullptr;
}

extern "C" dg_status dg_batch_destroy(dg_batch* b) {
  if (!b) return DG_OK;
  free_tables(b);
  int* pres[] = {b->d_pre_rows, b->d_pre_cols, b->d_pre_proj,
                 b->d_pre_bp,   b->d_pre_nlm,  b->d_pre_div};
  for (int* p : pres)
    if (p) (void)hipFree(p);
  // slices with one geometry share a plan: destroy each plan once
  for (size_t k = 0; k < b->plans.size(); ++k) {
    bool first = true;
    for (size_t e = 0; e < k && first; ++e) first = b->plans[e] != b->plans[k];
    if (first) dg_plan_destroy(b->plans[k]);
  }
  delete b;
  return DG_OK;
}

// Two acquisitions with the same parameters (the plan's tables depend on
// nothing else).
static bool same_geometry(const dg_geom& a, const dg_geom& b) {
  return a.kind == b.kind && a.n == b.n && a.n_views == b.n_views && a.n_bins == b.n_bins &&
         a.pixel_mm == b.pixel_mm && a.angle0_rad == b.angle0_rad && a.span_rad == b.span_rad &&
         a.bin_mm == b.bin_mm && a.dso_mm == b.dso_mm && a.ddo_mm == b.ddo_mm &&
         a.dgamma_rad == b.dgamma_rad;
}

extern "C" dg_status dg_batch_create(const dg_geom* geoms, int32_t n, dg_batch** out) {
  DG_ARG_CHECK(geoms && out && n >= 1 && n <= 4096, "dg_batch_create: bad arguments");
  dg_batch* b = new (std::nothrow) dg_batch();
  if (!b) {
    set_error("dg_batch_create: host allocation failed");
    return DG_ERR_NOMEM;
  }
  b->n = n;
  auto mk_prefix = [&](std::vector<int>& v) {
    v.assign(n + 1, 0);
  };
  mk_prefix(b->pre_rows);
  mk_prefix(b->pre_cols);
  mk_prefix(b->pre_proj);
  mk_prefix(b->pre_bp);
  mk_prefix(b->pre_nlm);
  mk_prefix(b->pre_div);
  b->img_off.assign(n + 1, 0);
  b->sino_off.assign(n + 1, 0);
  b->spec_off.assign(n + 1, 0);
  b->uniform_I = geoms[0].n;
  for (int s = 0; s < n; ++s) {
    // a slice whose geometry an earlier slice has uses that slice's plan, so
    // the kernels read one copy of its ray and view tables (C5's 16 slices
    // share one 4 MB fan-ray table instead of gathering from 16)
    dg_plan* p = nullptr;
    for (int e = 0; e < s && !p; ++e)
      if (same_geometry(geoms[e], geoms[s])) p = b->plans[e];
    if (!p) {
      dg_status rc = dg_plan_create(&geoms[s], &p);
      if (rc != DG_OK) {
        dg_batch_destroy(b);
        return rc;
      }
    }
    b->plans.push_back(p);
    if (!p->fft_ok) {
      dg_batch_destroy(b);
      set_error("dg_batch_create: a slice's image side is not supported by the FFT");
      return DG_ERR_UNSUPPORTED;
    }
    if (geoms[s].n != b->uniform_I) b->uniform_I = 0;
    const int kind_mode = geoms[s].kind == DG_GEOM_FAN ? 1 : 0;
    if (s == 0)
      b->bp_mode = kind_mode;
    else if (b->bp_mode != kind_mode)
      b->bp_mode = 2;
    const int I = p->I;
    b->img_off[s + 1] = b->img_off[s] + p->N;
    b->sino_off[s + 1] = b->sino_off[s] + p->M;
    b->spec_off[s + 1] = b->spec_off[s] + (int64_t)(I / 2 + 1) * I;
    b->pre_rows[s + 1] = b->pre_rows[s] + prec_row_blocks(I);
    b->pre_cols[s + 1] = b->pre_cols[s] + prec_col_blocks(I);
    b->pre_proj[s + 1] = b->pre_proj[s] + (int)project_blocks(p->M);
    b->pre_nlm[s + 1] = b->pre_nlm[s] + (int)nlm_blocks(I);
    b->pre_div[s + 1] = b->pre_div[s] + (int)red_grid(p->N);
  }
  // the back-projector's blocks per slice depend on the kernel the whole
  // batch runs (bp_mode)
  for (int s = 0; s < n; ++s)
    b->pre_bp[s + 1] = b->pre_bp[s] + (int)backproject_blocks(geoms[s].n, b->bp_mode);
  b->totN = b->img_off[n];
  b->totM = b->sino_off[n];
  b->totSpec = b->spec_off[n];
  dg_status rc;
  if ((rc = upload(b->pre_rows, &b->d_pre_rows)) != DG_OK ||
      (rc = upload(b->pre_cols, &b->d_pre_cols)) != DG_OK ||
      (rc = upload(b->pre_proj, &b->d_pre_proj)) != DG_OK ||
      (rc = upload(b->pre_bp, &b->d_pre_bp)) != DG_OK ||
      (rc = upload(b->pre_nlm, &b->d_pre_nlm)) != DG_OK ||
      (rc = upload(b->pre_div, &b->d_pre_div)) != DG_OK) {
    dg_batch_destroy(b);
    return rc;
  }
  *out = b;
  return DG_OK;
}

extern "C" dg_status dg_batch_layout(const dg_batch* b, int64_t* img_off, int64_t* sino_off) {
  DG_ARG_CHECK(b && img_off && sino_off, "dg_batch_layout: null argument");
  for (int s = 0; s <= b->n; ++s) {
    img_off[s] = b->img_off[s];
    sino_off[s] = b->sino_off[s];
  }
  return DG_OK;
}

extern "C" size_t dg_batch_workspace_bytes(const dg_batch* b) {
  return b ? batch_work_layout(b, nullptr, nullptr) : 0;
}

extern "C" dg_status dg_batch_bind(dg_batch* b, const float* y, const double* i0,
                                   const double* fro2, float* x, float* s, double* scal,
                                   float* mu_out, int32_t den_kind, const void* den_params,
                                   double eps_rel, void* work) {
  DG_ARG_CHECK(b && y && i0 && fro2 && x && s && scal && den_params && work,
               "dg_batch_bind: null argument");
  DG_ARG_CHECK(eps_rel > 0 && std::isfinite(eps_rel), "dg_batch_bind: eps_rel must be > 0");
  for (int k = 0; k < b->n; ++k) {
    DG_ARG_CHECK(i0[k] > 0 && std::isfinite(i0[k]) && fro2[k] > 0 && std::isfinite(fro2[k]),
                 "dg_batch_bind: i0 and fro2 must be positive");
    dg_status rc = den_kind == DG_DEN_CNN ? cnn_check_params(b->plans[k], den_params)
                                          : check_denoise_params(b->plans[k], den_kind, den_params);
    if (rc != DG_OK) return rc;
  }
  if (den_kind == DG_DEN_CNN && b->uniform_I == 0) {
    set_error("dg_batch_bind: the CNN denoiser needs slices of one image size");
    return DG_ERR_UNSUPPORTED;
  }
  if (den_kind == DG_DEN_HAAR || den_kind == DG_DEN_TV || den_kind == DG_DEN_TVW) {
    set_error("dg_batch_bind: batched runs support the NLM and CNN denoisers");
    return DG_ERR_UNSUPPORTED;
  }
  char* parts[12];
  batch_work_layout(b, work, parts);
  float2* spec = (float2*)parts[0];
  // slice k's mu at 2 img_off[k], its transpose right after it
  float* mu = (float*)parts[1];
  float* z = (float*)parts[3];
  float* g = (float*)parts[4];
  float* r = (float*)parts[5];
  float* xden = (float*)parts[6];
  float* xpert = (float*)parts[7];
  double* dpart = (double*)parts[8];
  float* fpart = (float*)parts[9];
  double* npart = (double*)parts[10];
  double* ppart = (double*)parts[11];
  const int n = b->n;
  std::vector<RowsFwdArgs> rf_x(n), rf_g(n);
  std::vector<ColsArgs> cols(n);
  std::vector<RowsInvArgs> ri_mu(n), ri_r(n), ri_out(n);
  std::vector<EpsArgs> eps(n);
  std::vector<ProjArgs> proj(n), projc(n);
  std::vector<ChanArgs> chan(n);
  std::vector<BpArgs> bp(n);
  std::vector<NlmArgs> nlm(n);
  std::vector<DivArgs> dv(n), dvn(n);
  const dg_nlm_params* np = (const dg_nlm_params*)den_params;
  for (int k = 0; k < n; ++k) {
    const dg_plan* p = b->plans[k];
    const int I = p->I;
    const int64_t io = b->img_off[k], so = b->sino_off[k];
    float2* sp = spec + b->spec_off[k];
    double* sc = scal + (size_t)k * DG_NSCAL;
    double* dp = dpart + (size_t)k * kPartMax;
    float* fp = fpart + (size_t)k * kPartMax;
    // with NLM, V^-1 x's first row workgroup finishes the previous
    // iteration's divergence step (from the NLM workgroups' partials)
    double* np_k = npart + b->pre_nlm[k];
    const int nb_k = b->pre_nlm[k + 1] - b->pre_nlm[k];
    rf_x[k] = RowsFwdArgs{x + io, sp, p->twiddle, I, 0, ChanArgs{},
                          den_kind == DG_DEN_NLM
                              ? DivFinish{np_k, nb_k, (double)p->N, sc + DG_S_EPS, sc}
                              : DivFinish{}};
    cols[k] = ColsArgs{sp, p->twiddle, I, 1};
    float* mu_k = mu + 2 * io;
    float* mu_t_k = mu_k + p->N;
    ri_mu[k] = RowsInvArgs{sp, p->twiddle, I, PREC_PLAIN, mu_k, mu_t_k, nullptr, nullptr,
                           nullptr};
    ri_r[k] = RowsInvArgs{sp, p->twiddle, I, PREC_UPDATE_R, r + io, nullptr, x + io, sc, fp};
    ri_out[k] = RowsInvArgs{sp, p->twiddle, I, PREC_PLAIN, mu_out ? mu_out + io : mu_k, nullptr,
                            nullptr, nullptr, nullptr};
    eps[k] = EpsArgs{fp, prec_row_blocks(I), eps_rel, sc + DG_S_EPS};
    // the output channel runs in the projector's epilogue (projc); proj is
    // the plain projector the autotuner times
    chan[k] = ChanArgs{p->M,    nullptr,  y + so,       s + so,       nullptr,
                       nullptr, sc,       nullptr,      i0[k],        fro2[k],
                       (double)p->N, ppart + b->pre_proj[k], b->pre_proj[k + 1] - b->pre_proj[k]};
    proj[k] = ProjArgs{p->rays, mu_k, mu_t_k, z + so, I, p->M, 0, ChanArgs{}};
    projc[k] = ProjArgs{p->rays, mu_k, mu_t_k, z + so, I, p->M, 1, chan[k]};
    // the channel finish runs in the slice's first row workgroup of V^-1 g
    rf_g[k] = RowsFwdArgs{g + io, sp, p->twiddle, I, 1, chan[k], DivFinish{}};
    bp[k] = BpArgs{p->rays, p->views, s + so, g + io, I, p->nv, p->nb,
                   p->g.kind == DG_GEOM_FAN ? 1 : 0, (float)p->half_diag_px, p->vrays, p->frays};
    // NLM also finishes the Monte-Carlo step and performs the divergence step
    if (den_kind == DG_DEN_NLM)
      nlm[k] = NlmArgs{r + io,           xden + io, xpert + io,       I,
                       np->search_radius, sc + DG_S_TAU_R, sc + DG_S_EPS, (float)np->hfac,
                       fp,               prec_row_blocks(I), eps_rel,   sc + DG_S_EPS,
                       x + io,           sc,        np_k};
    dv[k] = DivArgs{p->N, xden + io, xpert + io, x + io, sc + DG_S_EPS, nullptr, sc, dp,
                    b->pre_div[k + 1] - b->pre_div[k]};
    dvn[k] = DivArgs{p->N, xden + io, xpert + io, x + io, sc + DG_S_EPS, nullptr, sc, np_k, nb_k};
  }
  free_tables(b);
  dg_status rc;
  if ((rc = upload(rf_x, &b->t_rf_x)) != DG_OK || (rc = upload(rf_g, &b->t_rf_g)) != DG_OK ||
      (rc = upload(cols, &b->t_cols)) != DG_OK || (rc = upload(ri_mu, &b->t_ri_mu)) != DG_OK ||
      (rc = upload(ri_r, &b->t_ri_r)) != DG_OK || (rc = upload(ri_out, &b->t_ri_out)) != DG_OK ||
      (rc = upload(eps, &b->t_eps)) != DG_OK || (rc = upload(proj, &b->t_proj)) != DG_OK ||
      (rc = upload(projc, &b->t_projc)) != DG_OK ||
      (rc = upload(chan, &b->t_chan)) != DG_OK || (rc = upload(bp, &b->t_bp)) != DG_OK ||
      (rc = upload(nlm, &b->t_nlm)) != DG_OK || (rc = upload(dv, &b->t_div)) != DG_OK ||
      (rc = upload(dvn, &b->t_divn)) != DG_OK)
    return rc;
  b->x = x;
  b->s = s;
  b->scal = scal;
  b->y = y;
  b->mu_out = mu_out;
  b->r = r;
  b->xden = xden;
  b->xpert = xpert;
  b->den_kind = den_kind;
  if (den_kind == DG_DEN_NLM) {
    b->nlm = *np;
    b->h_nlm = nlm;
  }
  if (den_kind == DG_DEN_CNN) b->cnn = *(const dg_cnn_params*)den_params;
  b->bound = true;
  return DG_OK;
}

extern "C" dg_status dg_batch_state_init(dg_batch* b, double tau_x0, void* stream) {
  DG_ARG_CHECK(b && b->bound, "dg_batch_state_init: batch not bound");
  DG_ARG_CHECK(tau_x0 > 0 && std::isfinite(tau_x0), "dg_batch_state_init: tau_x0 must be > 0");
  hipStream_t st = (hipStream_t)stream;
  dg_status rc;
  if ((rc = launch_fill(b->x, b->totN, 0.0f, st)) != DG_OK) return rc;
  if ((rc = launch_fill(b->s, b->totM, 0.0f, st)) != DG_OK) return rc;
  hipLaunchKernelGGL(batch_init_scal, dim3((b->n * DG_NSCAL + 255) / 256), dim3(256), 0, st,
                     b->scal, b->n, tau_x0);
  DG_LAUNCH_CHECK("batch_init_scal");
  return DG_OK;
}

static dg_status batch_precondition(dg_batch* b, const RowsFwdArgs* rf, const RowsInvArgs* ri,
                                    int fin_t, double fin_eta, hipStream_t st) {
  const int n = b->n;
  dg_status rc;
  if ((rc = launch_prec_batch(0, rf, b->d_pre_rows, n, b->pre_rows[n], fin_t, fin_eta, st)) !=
      DG_OK)
    return rc;
  if ((rc = launch_prec_batch(1, b->t_cols, b->d_pre_cols, n, b->pre_cols[n], 0, 0.0, st)) !=
      DG_OK)
    return rc;
  return launch_prec_batch(2, ri, b->d_pre_rows, n, b->pre_rows[n], 0, 0.0, st);
}

extern "C" dg_status dgamp_batch_iterate(dg_batch* b, int32_t n_iter, int32_t t0,
                                         uint64_t probe_seed, double eta_x, double eta_s,
                                         int32_t onsager, int32_t channel_mode, int32_t write_mu,
                                         void* stream) {
  DG_ARG_CHECK(b && b->bound, "dgamp_batch_iterate: batch not bound");
  DG_ARG_CHECK(n_iter >= 0 && t0 >= 0, "dgamp_batch_iterate: bad iteration range");
  DG_ARG_CHECK(eta_x > 0 && eta_x <= 1 && eta_s > 0 && eta_s <= 1,
               "dgamp_batch_iterate: damping factors must be in (0, 1]");
  DG_ARG_CHECK(channel_mode == DG_CHANNEL_LAPLACE || channel_mode == DG_CHANNEL_MODE_ONLY,
               "dgamp_batch_iterate: unknown channel mode");
  hipStream_t st = (hipStream_t)stream;
  const int n = b->n;
  dg_status rc;
  const bool nlm = b->den_kind == DG_DEN_NLM;
  for (int it = 0; it < n_iter; ++it) {
    const int t = t0 + it;
    // (with NLM, also the scalar finish of iteration t - 1's divergence step)
    if ((rc = batch_precondition(b, b->t_rf_x, b->t_ri_mu, nlm && it > 0 ? t - 1 : -1, eta_x,
                                 st)) != DG_OK)
      return rc;
    // A with the output channel in its epilogue
    const ChanRun cr{channel_mode, onsager, t, eta_s};
    if ((rc = launch_project_batch(b->proj_variant, b->t_projc, b->d_pre_proj, n, b->pre_proj[n],
                                   cr, st)) != DG_OK)
      return rc;
    if ((rc = launch_backproject_batch(b->t_bp, b->d_pre_bp, n, b->pre_bp[n], b->bp_mode, st)) !=
        DG_OK)
      return rc;
    if ((rc = batch_precondition(b, b->t_rf_g, b->t_ri_r, t, eta_s, st)) != DG_OK) return rc;
    if (b->den_kind != DG_DEN_NLM &&
        (rc = launch_prec_batch(3, b->t_eps, nullptr, n, n, 0, 0.0, st)) != DG_OK)
      return rc;
    if (b->den_kind == DG_DEN_NLM) {
      // the divergence step runs inside the NLM launch
      rc = launch_nlm_batch(b->nlm.patch_radius, b->nlm_variant, b->t_nlm, b->d_pre_nlm, n,
                            b->pre_nlm[n], probe_seed, t, eta_x, t, st);
    } else {
      rc = cnn_launch_denoise_batch(&b->cnn, b->r, b->scal + DG_S_EPS, DG_NSCAL, probe_seed, t,
                                    b->xden, b->xpert, n, b->uniform_I, st);
      if (rc == DG_OK)
        rc = launch_div_batch(b->t_div, b->d_pre_div, n, b->pre_div[n], probe_seed, t, eta_x, t,
                              st);
    }
    if (rc != DG_OK) return rc;
  }
  const int t_last = nlm && n_iter > 0 ? t0 + n_iter - 1 : -1;
  if (write_mu) return batch_precondition(b, b->t_rf_x, b->t_ri_out, t_last, eta_x, st);
  if (t_last >= 0) return launch_div_finish_batch(b->t_divn, n, eta_x, t_last, st);
  return DG_OK;
}

// A whole batched reconstruction (state reset, n_iter iterations, mu_out when
// bound) captured as one graph.
extern "C" dg_status dg_batch_graph_create(dg_batch* b, double tau_x0, int32_t n_iter,
                                           uint64_t probe_seed, double eta_x, double eta_s,
                                           int32_t onsager, int32_t channel_mode,
                                           dg_graph** out) {
  DG_ARG_CHECK(b && b->bound && out, "dg_batch_graph_create: batch not bound");
  hipStream_t cs;
  DG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return hip_fail(e, "hipStreamBeginCapture");
  }
  dg_status rc = dg_batch_state_init(b, tau_x0, cs);
  if (rc == DG_OK)
    rc = dgamp_batch_iterate(b, n_iter, 0, probe_seed, eta_x, eta_s, onsager, channel_mode,
                             b->mu_out ? 1 : 0, cs);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (rc != DG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t exec;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(e, "hipGraphInstantiate");
  }
  *out = new dg_graph{graph, exec};
  return DG_OK;
}

// Autotuner: time each projector variant on the bound batch (or on a plan's
// own workspace image) and keep the fastest.
extern "C" dg_status dg_batch_autotune(dg_batch* b, int32_t reps, void* stream) {
  DG_ARG_CHECK(b && b->bound && reps >= 1, "dg_batch_autotune: batch not bound");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  DG_HIP(hipEventCreate(&e0));
  DG_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int best_v = b->proj_variant;
  dg_status rc = DG_OK;
  for (int v = 0; v < kProjNumVariants && rc == DG_OK; ++v) {
    rc = launch_project_batch(v, b->t_proj, b->d_pre_proj, b->n, b->pre_proj[b->n], ChanRun{},
                              st);  // warm
    if (rc != DG_OK) break;
    (void)hipEventRecord(e0, st);
    for (int k = 0; k < reps && rc == DG_OK; ++k)
      rc = launch_project_batch(v, b->t_proj, b->d_pre_proj, b->n, b->pre_proj[b->n], ChanRun{},
                                st);
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      best_v = v;
    }
  }
  if (rc == DG_OK && b->den_kind == DG_DEN_NLM && !b->h_nlm.empty()) {
    // the denoiser's variants on the bound slices, without the fused
    // divergence step (nothing of the iteration state is written) and with
    // fixed tau_r and eps in a scratch pair
    std::vector<NlmArgs> tn = b->h_nlm;
    double* d = nullptr;
    NlmArgs* dt = nullptr;
    const double sc[2] = {1e-4, 1e-3};
    hipError_t e;
    if ((e = hipMalloc(&d, sizeof(sc))) != hipSuccess ||
        (e = hipMalloc(&dt, sizeof(NlmArgs) * tn.size())) != hipSuccess) {
      rc = hip_fail(e, "dg_batch_autotune: hipMalloc");
    } else {
      for (NlmArgs& a : tn) {
        a.tau_r = d;
        a.eps = d + 1;
        a.eps_part = nullptr;
        a.eps_out = nullptr;
        a.x = nullptr;
        a.scal = nullptr;
        a.div_part = nullptr;
      }
      if ((e = hipMemcpy(d, sc, sizeof(sc), hipMemcpyHostToDevice)) != hipSuccess ||
          (e = hipMemcpy(dt, tn.data(), sizeof(NlmArgs) * tn.size(), hipMemcpyHostToDevice)) !=
              hipSuccess)
        rc = hip_fail(e, "dg_batch_autotune: hipMemcpy");
      float nbest = 1e30f;
      int nbest_v = b->nlm_variant;
      for (int v = 0; v < kNlmNumVariants && rc == DG_OK; ++v) {
        rc = launch_nlm_batch(b->nlm.patch_radius, v, dt, b->d_pre_nlm, b->n, b->pre_nlm[b->n], 0, 0,
                              0.0, 0, st);  // warm
        if (rc != DG_OK) break;
        (void)hipEventRecord(e0, st);
        for (int k = 0; k < reps && rc == DG_OK; ++k)
          rc = launch_nlm_batch(b->nlm.patch_radius, v, dt, b->d_pre_nlm, b->n, b->pre_nlm[b->n], 0,
                                0, 0.0, 0, st);
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < nbest) {
          nbest = ms;
          nbest_v = v;
        }
      }
      if (rc == DG_OK) {
        b->nlm_variant = nbest_v;
        for (dg_plan* p : b->plans) p->nlm_variant = nbest_v;
      }
    }
    if (dt) (void)hipFree(dt);
    if (d) (void)hipFree(d);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != DG_OK) return rc;
  b->proj_variant = best_v;
  for (dg_plan* p : b->plans) p->proj_variant = best_v;
  return DG_OK;
}

extern "C" int32_t dg_batch_nlm_variant(const dg_batch* b) { return b ? b->nlm_variant : -1; }

extern "C" dg_status dg_batch_set_nlm_variant(dg_batch* b, int32_t variant) {
  DG_ARG_CHECK(b && variant >= 0 && variant < kNlmNumVariants,
               "dg_batch_set_nlm_variant: bad argument");
  b->nlm_variant = variant;
  for (dg_plan* p : b->plans) p->nlm_variant = variant;
  return DG_OK;
}

extern "C" int32_t dg_batch_projector_variant(const dg_batch* b) { return b ? b->proj_variant : -1; }

extern "C" dg_status dg_batch_set_projector_variant(dg_batch* b, int32_t variant) {
  DG_ARG_CHECK(b && variant >= 0 && variant < kProjNumVariants,
               "dg_batch_set_projector_variant: bad argument");
  b->proj_variant = variant;
  for (dg_plan* p : b->plans) p->proj_variant = variant;
  return DG_OK;
}

extern "C" dg_status dg_plan_autotune(dg_plan* p, const float* img, const float* img_t,
                                      float* sino, int32_t reps, void* stream) {
  DG_ARG_CHECK(p && img && sino && reps >= 1, "dg_plan_autotune: null argument");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  DG_HIP(hipEventCreate(&e0));
  DG_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int best_v = p->proj_variant;
  dg_status rc = DG_OK;
  for (int v = 0; v < kProjNumVariants && rc == DG_OK; ++v) {
    ProjArgs A{p->rays, img, img_t, sino, p->I, p->M, 0, ChanArgs{}};
    rc = launch_project_variant(v, A, st);
    (void)hipEventRecord(e0, st);
    for (int k = 0; k < reps && rc == DG_OK; ++k) rc = launch_project_variant(v, A, st);
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      best_v = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != DG_OK) return rc;
  p->proj_variant = best_v;
  return DG_OK;
}

extern "C" int32_t dg_plan_projector_variant(const dg_plan* p) { return p ? p->proj_variant : -1; }

extern "C" dg_status dg_plan_set_projector_variant(dg_plan* p, int32_t variant) {
  DG_ARG_CHECK(p && variant >= 0 && variant < kProjNumVariants,
               "dg_plan_set_projector_variant: bad argument");
  p->proj_variant = variant;
  return DG_OK;
}
