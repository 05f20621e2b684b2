// D-GAMP-CT iteration driver (Algorithm 1, Sec. 4) and the Hutchinson
// estimate of ||A V^-1||_F^2 it needs.  One iteration is seven dependent
// steps, each a kernel (or the three passes of the preconditioner):
//   mu = V^-1 x  (row-major and transposed copies)   z = A mu
//   channel: tau_p, p = z - tau_p s, s, tau_s, tau_r  (one fused kernel)
//   g = A^T s    r = x + tau_r V^-1 g, eps = eps_rel max|r|  (fused epilogue)
//   D(r), D(r + eps b)  (one launch)   div, tau_x, damped x  (one kernel)
// All scalars stay on the device, so a whole run is host-sync free and can be
// captured into a graph by the caller.
#include <cmath>
#include <vector>

#include "dg_internal.h"

namespace dg {

dg_status check_denoise_params(const dg_plan* p, int kind, const void* params);
dg_status launch_denoiser(const dg_plan* p, int kind, const void* params, const float* r,
                          const double* tau_r, const double* eps, uint64_t seed, int iter,
                          float* x_den, float* x_pert, hipStream_t st, const EpsFinish* ef,
                          const DivFuse* df);
unsigned int nlm_blocks(int I);
unsigned int project_blocks(int64_t M);
dg_status launch_project_run(int variant, const ProjArgs& A, const ChanRun& cr, hipStream_t s);
dg_status launch_div_finish(const DivArgs& A, double eta_x, int t, hipStream_t st);
int prec_row_blocks(int I);
dg_status launch_div(const dg_plan* p, const float* xden, const float* xpert, float* x,
                     const double* eps, double* div_out, double* scal, int mode, uint64_t seed,
                     int iter, double eta_x, int t, double* partials, hipStream_t st);
dg_status launch_probe(float* b, int64_t N, uint64_t seed, int k, hipStream_t st);
size_t denoise_work_bytes(const dg_plan* p);
unsigned int red_grid(int64_t N);
dg_status cnn_check_params(const dg_plan* p, const void* params);
dg_status cnn_launch_denoise(const dg_plan* p, const void* params, const float* r,
                             const double* eps, uint64_t seed, int iter, float* x_den,
                             float* x_pert, double* div_dot_out, hipStream_t st);

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static constexpr int kMaxBlocks = 1024;

struct IterWork {
  double* dpart;
  double* npart;  // divergence partials of the NLM workgroups
  float* fpart;
  float *mu, *mu_t, *z, *g, *r, *xden, *xpert;
  float2* spec;
};

static size_t iter_work_layout(const dg_plan* p, void* base, IterWork* w) {
  char* c = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* ptr = c ? c + off : nullptr;
    off += align256(bytes);
    return ptr;
  };
  IterWork t;
  // per-workgroup FP64 partials: the projector's (fused channel), the
  // divergence pass's
  const size_t np = project_blocks(p->M);
  t.dpart = (double*)take(sizeof(double) * (np > (size_t)kMaxBlocks ? np : (size_t)kMaxBlocks));
  t.npart = (double*)take(sizeof(double) * nlm_blocks(p->I));
  t.fpart = (float*)take(sizeof(float) * kMaxBlocks);
  const size_t nb = sizeof(float) * (size_t)p->N, mb = sizeof(float) * (size_t)p->M;
  t.mu = (float*)take(nb);
  t.mu_t = (float*)take(nb);
  t.z = (float*)take(mb);
  t.g = (float*)take(nb);
  t.r = (float*)take(nb);
  t.xden = (float*)take(nb);
  t.xpert = (float*)take(nb);
  t.spec = (float2*)take(precond_work_bytes(p));
  if (w) *w = t;
  return off;
}

__global__ void fill_f32(float* p, int64_t n, float v) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    p[k] = v;
}

__global__ void init_scal(double* scal, double tau_x0) {
  int k = threadIdx.x;
  if (k < DG_NSCAL) scal[k] = (k == DG_S_TAU_X) ? tau_x0 : 0.0;
}

__global__ void log_copy(const double* scal, double* log) {
  if (threadIdx.x == 0) {
    log[0] = scal[DG_S_TAU_P];
    log[1] = scal[DG_S_TAU_S];
    log[2] = scal[DG_S_TAU_R];
    log[3] = scal[DG_S_DIV];
    log[4] = scal[DG_S_TAU_X];
    log[5] = scal[DG_S_EPS];
    log[6] = scal[DG_S_STATUS];
    log[7] = scal[DG_S_CLAMPS];
  }
}

// per-block partial sums of z^2 (FP64)
__global__ void __launch_bounds__(256)
sumsq_partial(const float* __restrict__ z, int64_t n, double* __restrict__ partials) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
    double v = z[k];
    acc += v * v;
  }
  double bs = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// out += scale * sum(partials)
__global__ void __launch_bounds__(256)
sumsq_finish(const double* __restrict__ partials, int nblk, double scale, double* out) {
  __shared__ double red[4];
  const double tot = finish_sum(partials, nblk, red);
  if (threadIdx.x == 0) *out += tot * scale;
}

__global__ void set_f64(double* p, double v) {
  if (threadIdx.x == 0) *p = v;
}

dg_status launch_fill(float* p, int64_t n, float v, hipStream_t st) {
  hipLaunchKernelGGL(fill_f32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, n, v);
  DG_LAUNCH_CHECK("fill_f32");
  return DG_OK;
}

size_t iter_work_bytes(const dg_plan* p) { return iter_work_layout(p, nullptr, nullptr); }
size_t se_work_bytes(const dg_plan* p);

}  // namespace dg

using namespace dg;

extern "C" size_t dg_workspace_bytes(const dg_plan* p, int32_t op) {
  if (!p) return 0;
  switch (op) {
    case DG_OP_PRECOND:
      return precond_work_bytes(p);
    case DG_OP_DENOISE:
      return denoise_work_bytes(p);
    case DG_OP_DGAMP:
    case DG_OP_FRO2:
      return iter_work_bytes(p);
    case DG_OP_SE:
      return se_work_bytes(p);
    default:
      return 0;
  }
}

extern "C" dg_status dgamp_state_init(const dg_plan* p, dgamp_state* st, double tau_x0,
                                      void* stream) {
  DG_ARG_CHECK(p && st && st->x && st->s && st->scal, "dgamp_state_init: null argument");
  DG_ARG_CHECK(tau_x0 > 0 && std::isfinite(tau_x0), "dgamp_state_init: tau_x0 must be > 0");
  hipStream_t s = (hipStream_t)stream;
  dg_status rc;
  if ((rc = launch_fill(st->x, p->N, 0.0f, s)) != DG_OK) return rc;
  if ((rc = launch_fill(st->s, p->M, 0.0f, s)) != DG_OK) return rc;
  hipLaunchKernelGGL(init_scal, dim3(1), dim3(64), 0, s, st->scal, tau_x0);
  DG_LAUNCH_CHECK("init_scal");
  st->t = 0;
  return DG_OK;
}

extern "C" dg_status dgamp_iterate(const dg_plan* p, const float* y, const dgamp_opts* o,
                                   dgamp_state* st, float* mu_out, double* log, void* work,
                                   void* stream) {
  DG_ARG_CHECK(p && y && o && st && work, "dgamp_iterate: null argument");
  DG_ARG_CHECK(st->x && st->s && st->scal, "dgamp_iterate: state buffers missing");
  DG_ARG_CHECK(o->n_iter >= 0 && o->n_iter <= 100000, "dgamp_iterate: bad n_iter");
  DG_ARG_CHECK(o->fro2 > 0 && std::isfinite(o->fro2), "dgamp_iterate: fro2 must be > 0");
  DG_ARG_CHECK(o->i0 > 0 && std::isfinite(o->i0), "dgamp_iterate: i0 must be > 0");
  DG_ARG_CHECK(o->eps_rel > 0 && std::isfinite(o->eps_rel), "dgamp_iterate: eps_rel must be > 0");
  DG_ARG_CHECK(o->eta_x > 0 && o->eta_x <= 1 && o->eta_s > 0 && o->eta_s <= 1,
               "dgamp_iterate: damping factors must be in (0, 1]");
  DG_ARG_CHECK(o->channel_mode == DG_CHANNEL_LAPLACE || o->channel_mode == DG_CHANNEL_MODE_ONLY,
               "dgamp_iterate: unknown channel mode");
  if (!p->fft_ok) {
    set_error("dgamp_iterate: image side not supported by the preconditioner FFT");
    return DG_ERR_UNSUPPORTED;
  }
  dg_status rc = (o->den_kind == DG_DEN_CNN) ? cnn_check_params(p, o->den_params)
                                             : check_denoise_params(p, o->den_kind, o->den_params);
  if (rc != DG_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  IterWork w;
  iter_work_layout(p, work, &w);
  const double N = (double)p->N;
  hipEvent_t* ev = (hipEvent_t*)o->phase_events;
  const uint32_t pmask = o->phase_mask;
  auto mark = [&](int it, int k) -> dg_status {
    if (ev && (pmask == 0 || ((pmask >> k) & 1u)))
      DG_HIP(hipEventRecord(ev[(size_t)it * (DG_NPHASES + 1) + k], s));
    return DG_OK;
  };
  const bool nlm = o->den_kind == DG_DEN_NLM;
  // with NLM the divergence step's scalar finish of iteration t runs in the
  // finish workgroup of the next V^-1 x's row pass (or of the final V^-1 x
  // for mu_out, or in a finish launch of its own after the last iteration)
  const DivFinish pending{w.npart, (int)nlm_blocks(p->I), N, st->scal + DG_S_EPS, st->scal};
  auto log_it = [&](int it) -> dg_status {
    if (log) {
      hipLaunchKernelGGL(log_copy, dim3(1), dim3(64), 0, s, st->scal,
                         log + (size_t)it * DG_LOG_STRIDE);
      DG_LAUNCH_CHECK("log_copy");
    }
    return DG_OK;
  };
  for (int it = 0; it < o->n_iter; ++it) {
    const int t = st->t + it;
    if ((rc = mark(it, 0)) != DG_OK) return rc;
    PrecArgs a{};
    a.in = st->x;
    a.out = w.mu;
    a.out_t = w.mu_t;
    a.spec = w.spec;
    a.dir = 1;
    a.epilogue = PREC_PLAIN;
    a.fin_t = -1;
    if (nlm && it > 0) {
      a.dv = pending;
      a.fin_t = t - 1;
      a.fin_eta = o->eta_x;
    }
    if ((rc = launch_precondition(p, a, s)) != DG_OK) return rc;
    if (nlm && it > 0 && (rc = log_it(it - 1)) != DG_OK) return rc;
    if ((rc = mark(it, 1)) != DG_OK) return rc;
    // A with the output channel applied to every ray in the same launch; the
    // channel's finish (tau_s, tau_r) runs in the finish workgroup of the
    // next preconditioner application's row pass, and NLM finishes the MC step
    const ChanArgs chan{p->M, nullptr, y,      st->s,   nullptr, nullptr, st->scal,
                        nullptr, o->i0, o->fro2, N, w.dpart, (int)project_blocks(p->M)};
    const ProjArgs pa{p->rays, w.mu, w.mu_t, w.z, p->I, p->M, 1, chan};
    const ChanRun cr{o->channel_mode, o->onsager, t, o->eta_s};
    if ((rc = launch_project_run(p->proj_variant, pa, cr, s)) != DG_OK) return rc;
    if ((rc = mark(it, 2)) != DG_OK) return rc;
    if ((rc = mark(it, 3)) != DG_OK) return rc;
    if ((rc = launch_backproject(p, st->s, w.g, s)) != DG_OK) return rc;
    if ((rc = mark(it, 4)) != DG_OK) return rc;
    PrecArgs b{};
    b.in = w.g;
    b.out = w.r;
    b.out_t = nullptr;
    b.spec = w.spec;
    b.dir = 1;
    b.epilogue = PREC_UPDATE_R;
    b.x = st->x;
    b.scal = st->scal;
    b.scal_out = st->scal;
    b.eps_rel = o->eps_rel;
    b.partials = w.fpart;
    b.eps_elsewhere = nlm ? 1 : 0;
    b.fin = 1;
    b.chan = chan;
    b.fin_eta = o->eta_s;
    b.fin_t = t;
    if ((rc = launch_precondition(p, b, s)) != DG_OK) return rc;
    if ((rc = mark(it, 5)) != DG_OK) return rc;
    const double* tau_r = st->scal + DG_S_TAU_R;
    const double* eps = st->scal + DG_S_EPS;
    const EpsFinish ef{w.fpart, prec_row_blocks(p->I), o->eps_rel, st->scal + DG_S_EPS};
    const DivFuse df{st->x, st->scal, w.npart, o->eta_x, t};
    if (o->den_kind == DG_DEN_CNN)
      rc = cnn_launch_denoise(p, o->den_params, w.r, eps, o->probe_seed, t, w.xden, w.xpert,
                              nullptr, s);
    else
      rc = launch_denoiser(p, o->den_kind, o->den_params, w.r, tau_r, eps, o->probe_seed, t,
                           w.xden, w.xpert, s, nlm ? &ef : nullptr, nlm ? &df : nullptr);
    if (rc != DG_OK) return rc;
    if ((rc = mark(it, 6)) != DG_OK) return rc;
    // NLM performs the divergence step's per-pixel part in its own launch
    if (!nlm) {
      if ((rc = launch_div(p, w.xden, w.xpert, st->x, eps, nullptr, st->scal, 1, o->probe_seed, t,
                           o->eta_x, t, w.dpart, s)) != DG_OK)
        return rc;
      if ((rc = log_it(it)) != DG_OK) return rc;
    }
    if ((rc = mark(it, 7)) != DG_OK) return rc;
  }
  const int t_last = st->t + o->n_iter - 1;
  const bool finish = nlm && o->n_iter > 0;
  st->t += o->n_iter;
  if (mu_out) {
    PrecArgs a{};
    a.in = st->x;
    a.out = mu_out;
    a.spec = w.spec;
    a.dir = 1;
    a.epilogue = PREC_PLAIN;
    a.fin_t = -1;
    if (finish) {
      a.dv = pending;
      a.fin_t = t_last;
      a.fin_eta = o->eta_x;
    }
    if ((rc = launch_precondition(p, a, s)) != DG_OK) return rc;
  } else if (finish) {
    const DivArgs A{p->N, w.xden, w.xpert, st->x, st->scal + DG_S_EPS, nullptr, st->scal,
                    w.npart, (int)nlm_blocks(p->I)};
    if ((rc = launch_div_finish(A, o->eta_x, t_last, s)) != DG_OK) return rc;
  }
  if (finish && (rc = log_it(o->n_iter - 1)) != DG_OK) return rc;
  return DG_OK;
}

extern "C" dg_status dg_check_status(const double* scal, int32_t n_slices, int32_t* failed_slice,
                                     int32_t* failed_iter, void* stream) {
  DG_ARG_CHECK(scal && n_slices >= 1, "dg_check_status: null scalars or no slices");
  DG_HIP(hipStreamSynchronize((hipStream_t)stream));
  std::vector<double> h((size_t)n_slices * DG_NSCAL);
  DG_HIP(hipMemcpy(h.data(), scal, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
  if (failed_slice) *failed_slice = -1;
  if (failed_iter) *failed_iter = -1;
  for (int32_t k = 0; k < n_slices; ++k) {
    const double v = h[(size_t)k * DG_NSCAL + DG_S_STATUS];
    if (v != 0.0) {
      const int32_t it = (int32_t)v - 1;
      if (failed_slice) *failed_slice = k;
      if (failed_iter) *failed_iter = it;
      set_error("slice " + std::to_string(k) + ": a GAMP variance became non-finite or "
                "non-positive at iteration " + std::to_string(it) +
                "; later iterations left its state unchanged");
      return DG_ERR_NUMERIC;
    }
  }
  return DG_OK;
}

extern "C" dg_status dg_fro2_hutchinson(const dg_plan* p, int32_t n_probes, uint64_t seed,
                                        double* out, void* work, void* stream) {
  DG_ARG_CHECK(p && out && work, "dg_fro2_hutchinson: null argument");
  DG_ARG_CHECK(n_probes >= 1, "dg_fro2_hutchinson: n_probes must be >= 1");
  if (!p->fft_ok) {
    set_error("dg_fro2_hutchinson: image side not supported by the preconditioner FFT");
    return DG_ERR_UNSUPPORTED;
  }
  hipStream_t s = (hipStream_t)stream;
  IterWork w;
  iter_work_layout(p, work, &w);
  dg_status rc;
  hipLaunchKernelGGL(set_f64, dim3(1), dim3(64), 0, s, out, 0.0);
  DG_LAUNCH_CHECK("set_f64");
  for (int k = 0; k < n_probes; ++k) {
    if ((rc = launch_probe(w.r, p->N, seed, k, s)) != DG_OK) return rc;
    PrecArgs a{};
    a.in = w.r;
    a.out = w.mu;
    a.out_t = w.mu_t;
    a.spec = w.spec;
    a.dir = 1;
    a.epilogue = PREC_PLAIN;
    if ((rc = launch_precondition(p, a, s)) != DG_OK) return rc;
    if ((rc = launch_project(p, w.mu, w.mu_t, w.z, s)) != DG_OK) return rc;
    const unsigned int g = red_grid(p->M);
    hipLaunchKernelGGL(sumsq_partial, dim3(g), dim3(256), 0, s, w.z, p->M, w.dpart);
    DG_LAUNCH_CHECK("sumsq_partial");
    hipLaunchKernelGGL(sumsq_finish, dim3(1), dim3(256), 0, s, w.dpart, (int)g, 1.0 / n_probes, out);
    DG_LAUNCH_CHECK("sumsq_finish");
  }
  return DG_OK;
}

extern "C" dg_status dgamp_graph_create(const dg_plan* p, const float* y, const dgamp_opts* o,
                                        dgamp_state* st, double tau_x0, float* mu_out,
                                        double* log, void* work, dg_graph** out) {
  DG_ARG_CHECK(p && y && o && st && work && out, "dgamp_graph_create: null argument");
  DG_ARG_CHECK(o->phase_events == nullptr, "dgamp_graph_create: phase events cannot be captured");
  hipStream_t cs;
  DG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  const int32_t t_before = st->t;
  dg_status rc = DG_OK;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return hip_fail(e, "hipStreamBeginCapture");
  }
  if (tau_x0 > 0) rc = dgamp_state_init(p, st, tau_x0, cs);
  if (rc == DG_OK) rc = dgamp_iterate(p, y, o, st, mu_out, log, work, cs);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  st->t = t_before;
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
  dg_graph* g = new dg_graph{graph, exec};
  *out = g;
  return DG_OK;
}

extern "C" dg_status dg_graph_launch(dg_graph* g, void* stream) {
  DG_ARG_CHECK(g != nullptr, "dg_graph_launch: null graph");
  DG_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return DG_OK;
}

extern "C" dg_status dg_graph_destroy(dg_graph* g) {
  if (!g) return DG_OK;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
  return DG_OK;
}
