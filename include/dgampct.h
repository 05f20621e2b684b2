/*
 * dgampct.h -- C ABI of the D-GAMP-CT hot path on AMD Instinct MI355X (gfx950).
 *
 * Method: Perelli, Lexa, Can & Davies, "Compressive CT reconstruction through
 * Denoising Approximate Message Passing" (arXiv 1609.04661).  Each entry point
 * cites the passage that defines the operation it computes.
 *
 * Conventions shared by every call
 *   - Image: I x I, row-major, row 0 on top, FP32; pixel (i, j) has centre
 *     ((j - (I-1)/2) h, ((I-1)/2 - i) h) in mm.
 *   - Sinogram: view-major [n_views][n_bins], FP32; ray index = k*n_bins + b.
 *   - Every array pointer is DEVICE memory owned by the caller unless stated;
 *     the library never frees caller memory and keeps no pointer after return.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = legacy default
 *     stream).  Outputs are overwritten, never accumulated into.
 *   - Arguments are validated on the host before anything is launched; a bad
 *     argument returns DG_ERR_ARG with nothing launched, dg_last_error() gives
 *     the reason (thread-local text).
 *   - Scalars that feed the next step (tau_p, tau_s, tau_r, div, ...) live in
 *     device memory, so a T-iteration loop needs no host synchronisation.
 *   - A plan may be used by several calls on one stream; concurrent calls on
 *     different streams need separate workspaces.
 */
#ifndef DGAMPCT_H
#define DGAMPCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dg_status;
#define DG_OK 0
#define DG_ERR_ARG (-1)         /* invalid argument: nothing launched          */
#define DG_ERR_HIP (-2)         /* HIP runtime error (message in dg_last_error)*/
#define DG_ERR_NUMERIC (-3)     /* a GAMP variance became non-finite or <= 0   */
                                /* (reported by dg_check_status: the iteration */
                                /* calls are asynchronous and record it in the */
                                /* device status word scal[DG_S_STATUS])       */
#define DG_ERR_UNSUPPORTED (-4) /* size or option not implemented              */
#define DG_ERR_NOMEM (-5)       /* device allocation failed (plan tables only)  */

#define DG_GEOM_PARALLEL 0
#define DG_GEOM_FAN 1

/* One acquisition (Sec. 2.1, eqs. linCT and Phi_mtx: one system-matrix row per
 * measured ray, J = n_bins * n_views rows; only measured views are listed).
 *   parallel: theta_k = angle0 + k*span/n_views (end point excluded), ray b is
 *     the line <u, (cos theta_k, sin theta_k)> = (b - (n_bins-1)/2) * bin_mm.
 *   fan (equiangular arc detector): source at dso*(cos beta_k, sin beta_k),
 *     beta_k = angle0 + k*span/n_views; ray b leaves the source towards the
 *     iso-centre rotated by gamma_b = (b - (n_bins-1)/2) * dgamma; dgamma = 0
 *     picks the pitch whose fan covers the circle circumscribing the image.
 *     ddo_mm is recorded but does not change the ray lines.
 * Angles that are exact multiples of pi/2 use exact trig values.             */
typedef struct dg_geom {
  int32_t kind;       /* DG_GEOM_PARALLEL or DG_GEOM_FAN                 */
  int32_t n;          /* image side I, 8 <= I <= 4096                     */
  int32_t n_views;    /* N_theta >= 1                                     */
  int32_t n_bins;     /* N_dec >= 1                                       */
  double pixel_mm;    /* h > 0                                            */
  double angle0_rad;
  double span_rad;
  double bin_mm;      /* parallel detector pitch > 0, with sqrt(2) h/bin_mm
                         (1.5 I + 1) + n_bins / 2 + 8 < 65536 (bin coordinates
                         over the image stay below 2^16)                   */
  double dso_mm;      /* fan: source to iso-centre, > I*h/sqrt(2)         */
  double ddo_mm;      /* fan: iso-centre to detector                      */
  double dgamma_rad;  /* fan: angular bin pitch, 0 = cover the image       */
} dg_geom;

typedef struct dg_plan dg_plan; /* geometry tables, FFT twiddles (device)   */

/* Build the per-ray line tables, the FFT tables and the preconditioner
 * symbol for `g` on the current HIP device.  Synchronous.  The plan owns its
 * (read-only) device tables until dg_plan_destroy.  A geometry outside the
 * limits stated in dg_geom returns DG_ERR_ARG with a message.              */
dg_status dg_plan_create(const dg_geom* g, dg_plan** out);
dg_status dg_plan_destroy(dg_plan* plan);

/* Workspace (device bytes) an operation needs with this plan.               */
#define DG_OP_PRECOND 0
#define DG_OP_DENOISE 1
#define DG_OP_DGAMP 2
#define DG_OP_FRO2 3
#define DG_OP_SE 4
size_t dg_workspace_bytes(const dg_plan* plan, int32_t op);
/* Workspace of gamp_poisson_out for m rays.                                 */
size_t dg_channel_workspace_bytes(int64_t m);

const char* dg_last_error(void);

/* z = A mu: exact chord lengths of each ray through each pixel (Sec. 2.1,
 * eqs. paramdiscrete and linCT; the pixel indicator basis).  A line lying
 * exactly on a pixel edge gives half of its length to each neighbour.
 * img: I*I floats; sino: n_views*n_bins floats (mm * 1/mm = dimensionless).
 * img_t: optional transposed copy of img (img_t[j*I+i] = img[i*I+j]) that
 * makes the reads of near-horizontal rays coalesced.  NULL: no copy is made
 * and those rays read img with a stride of I floats, several times slower
 * (512^2, 64 views: about 88 us against 16 us).  The sinogram is the same
 * bit for bit either way, wherever img_t lies in memory.                    */
dg_status ct_project(const dg_plan* plan, const float* img, const float* img_t,
                     float* sino, void* stream);

/* g = A^T s with the same weights as ct_project (exact adjoint up to FP32
 * rounding), computed as a gather per pixel (no atomics, deterministic).   */
dg_status ct_backproject(const dg_plan* plan, const float* sino, float* img,
                         void* stream);

/* Fourier-slice Radon operator (Sec. 2.4, eq. Radon_op: A = F_gamma^-1
 * Omega F), the paper's O(N log N) operator model, for parallel-beam
 * geometries: the image as point masses h^2 mu_ij at the pixel centres of
 * the ray-driven grid; view k samples its 2D Fourier transform along
 * rho (cos theta_k, sin theta_k) at rho_m = (m - floor(n_bins/2)) /
 * (n_bins bin_mm), m < n_bins, and the radial inverse DFT returns
 *   sino_k(b) = Re (1/(n_bins bin_mm)) sum_m P_k(m) exp(2 pi i rho_m s_b),
 *   s_b = (b - (n_bins - 1)/2) bin_mm
 * (line integrals of the band-limited image; a unit pixel at the origin
 * gives h at the central bin when bin_mm = h).  Computed as a non-uniform
 * FFT: deapodised image on a 2I x 2I grid, 2D FFT, Kaiser-Bessel
 * interpolation of width 8 at the polar samples (relative error ~1e-8
 * before FP32 rounding), direct radial DFT.  ct_backproject_fourier is its
 * exact adjoint (the transposed steps; a deterministic gather onto the grid).
 * The operator object holds the interpolation weights and the adjoint's
 * sparse table (about 8 * 81 * n_views * n_bins bytes) on the current device.
 * Image side: a power of two in [8, 512]; n_bins >= 2, n_views * n_bins
 * <= 2^22 (else DG_ERR_ARG).  img: I*I floats, sino:
 * n_views*n_bins floats (view-major), work: dg_fourier_workspace_bytes.    */
typedef struct dg_fourier dg_fourier;
dg_status dg_fourier_create(const dg_geom* g, dg_fourier** out);
dg_status dg_fourier_destroy(dg_fourier* f);
size_t dg_fourier_workspace_bytes(const dg_fourier* f);
dg_status ct_project_fourier(const dg_fourier* f, const float* img, float* sino, void* work,
                             void* stream);
dg_status ct_backproject_fourier(const dg_fourier* f, const float* sino, float* img, void* work,
                                 void* stream);

/* Cone preconditioner (Sec. 2.4, eq. PPFT preconditioner; eq. Aprecon):
 * V = F^-1 C^(1/2) F with C = diag(1/|rho|) on the unpadded I x I DFT grid,
 * |rho| in cycles per pixel, DC value 4 ln(1+sqrt 2) I (the mean of 1/|rho|
 * over the central DFT cell).
 *   dir = +1: out = V^-1 in  (x -> mu, multiplies the spectrum by |rho|^1/2)
 *   dir = -1: out = V in     (mu -> x)
 * in/out: I*I floats (may alias); work: dg_workspace_bytes(DG_OP_PRECOND).
 * I must be 2^a * 3^b with b <= 1, 8 <= I <= 1024 (DG_ERR_UNSUPPORTED).      */
dg_status ct_precondition(const dg_plan* plan, int32_t dir, const float* in, float* out,
                          void* work, void* stream);

/* GAMP output channel for Poisson transmission data (Sec. 4.2 eqs. noise_mod,
 * MMSEmm, post_exp; Appendix A; Algorithm 1 step 2):
 *   posterior of z ~ exp(-(z-p)^2/(2 tau_p) - y z - i0 e^-z),
 *   s_i = (E[z_i] - p_i)/tau_p,  *tau_s = sum_i (1 - Var[z_i]/tau_p) / (m tau_p)
 * with E and Var from the Laplace expansion around the mode (mode = 0:
 * second-order fully exponential form, Var clamped to [0, tau_p];
 * mode = 1: E = mode, Var = curvature^-1).
 * p, y, s_out: m floats (y holds counts); tau_p, tau_s_out: one device double.
 * work: dg_channel_workspace_bytes(m).  tau_s is reduced in FP64.           */
#define DG_CHANNEL_LAPLACE 0
#define DG_CHANNEL_MODE_ONLY 1
dg_status gamp_poisson_out(int64_t m, const float* p, const float* y, const double* tau_p,
                           double i0, int32_t mode, float* s_out, double* tau_s_out,
                           void* work, void* stream);

/* Plug-in denoiser x = D(r) and its Monte-Carlo divergence (Sec. 4.3, eqs.
 * rGAMP, D_in, MC_SURE):
 *   div = b^T (D(r + eps b) - D(r)) / (N eps),  eps = max(eps_rel max|r|, 1e-12),
 *   b_i = 1 - 2 (SplitMix64(probe_seed ^ (iter << 32) ^ i) & 1)   (one probe).
 * kind/params (host pointer to the struct below):
 *   DG_DEN_HAAR: orthonormal 2D Haar pyramid, soft threshold alpha*sqrt(tau_r)
 *                on detail coefficients (I <= 512, levels = log2 I - 2 by default)
 *   DG_DEN_NLM : non-local means, sigma = sqrt(tau_r)
 *   DG_DEN_CNN : residual CNN (see dg_cnn_params)
 *   DG_DEN_TV  : proximal isotropic total variation (Sec. 6, "Proximal-based TV
 *                denoiser"): argmin_x 1/2 ||x - r||^2 + lam TV(x), lam = alpha
 *                sqrt(tau_r), forward differences with zero difference past the
 *                last row / column, as `iters` fast gradient projection steps on
 *                the dual (Beck & Teboulle 2009) from a zero dual; the map is
 *                those steps.  work: device, dg_tv_workspace_bytes(I*I) bytes,
 *                owned by the caller, overwritten by every call.
 *   DG_DEN_TVW : the same map in the (V^T V)^-1 metric (Sec. 4.3 and Sec. 6 name
 *                it for input in the preconditioned domain): argmin_x 1/2
 *                (x - r)^T W (x - r) + lam TV(x), W = (V^T V)^-1 the circulant
 *                with symbol 1/c (c the cone symbol of ct_precondition; with
 *                metric = 1, W = V^T V, symbol c, the figure's reading), lam =
 *                alpha sqrt(tau_r), as `iters` Chambolle-Pock primal-dual steps
 *                (sigma = tau = 1/(lam sqrt 8), theta = 1) from x = r and a zero
 *                dual, each with a Fourier-domain primal step; the map is those
 *                steps.  Params: dg_tv_params with work of
 *                dg_tvw_workspace_bytes(I) bytes (device, caller-owned,
 *                overwritten by every call).  The side I must be one the FFT
 *                supports (2^a or 3 * 2^a, <= 1024), else DG_ERR_ARG.
 *   DG_DEN_BM3D: two-stage block-matching 3D filter (the paper's denoiser,
 *                Dabov et al. 2007): 8x8 blocks on a step-3 grid, groups of
 *                the reference block and up to 15 others within +-19 pixels
 *                with mean squared difference <= 4.8 sigma^2 (by distance,
 *                then raster position; a power of two), 8x8 DCT + Haar along
 *                the group, hard threshold 2.7 sigma with 1/(sigma^2 N_har)
 *                weights, then the Wiener stage on the same groups with
 *                1/(sigma^2 ||W||^2) weights (1 where every factor vanishes),
 *                Kaiser-window (beta 2)
 *                aggregation; sigma = sqrt(tau_r).  The decisions (distances,
 *                threshold tests) are FP32 in a fixed order; the aggregation
 *                sums by FP32 atomics (reproducible to rounding, not bit for
 *                bit).  Params: dg_bm3d_params with work of
 *                dg_bm3d_workspace_bytes(I) bytes (device, caller-owned,
 *                overwritten by every call); 16 <= I <= 4096.
 * r, x_out: I*I floats; tau_r: device double; div_out: device double or NULL
 * (NULL skips the probe evaluation).  work: dg_workspace_bytes(DG_OP_DENOISE). */
#define DG_DEN_HAAR 0
#define DG_DEN_NLM 1
#define DG_DEN_CNN 2
#define DG_DEN_TV 3
#define DG_DEN_TVW 4
#define DG_DEN_BM3D 5
typedef struct dg_haar_params { double alpha; int32_t levels; /* 0 = log2 I - 2 */ } dg_haar_params;
typedef struct dg_nlm_params { int32_t patch_radius; int32_t search_radius; double hfac; } dg_nlm_params;
typedef struct dg_cnn_params {
  const void* weights;  /* device: packed network, dg_cnn_weight_bytes() bytes   */
  void* work;           /* device: dg_cnn_workspace_bytes(I*I) bytes (activations) */
} dg_cnn_params;
typedef struct dg_tv_params {
  double alpha;    /* lam = alpha * sqrt(tau_r), >= 0                            */
  int32_t iters;   /* TV: fast gradient projection steps; TVW: primal-dual       */
                   /* steps; 1 .. 10000                                          */
  int32_t metric;  /* TVW only: 0 = W = (V^T V)^-1 (the norm the text names),    */
                   /* 1 = W = V^T V (the subscript of the paper's TV figure);    */
                   /* TV ignores it                                              */
  void* work;      /* device: dg_tv_workspace_bytes(I*I) bytes for TV,           */
                   /* dg_tvw_workspace_bytes(I) for TVW                          */
} dg_tv_params;
typedef struct dg_bm3d_params {
  void* work;      /* device: dg_bm3d_workspace_bytes(I) bytes                  */
} dg_bm3d_params;
/* Work bytes of DG_DEN_BM3D for an I x I image (0 for side < 8). */
size_t dg_bm3d_workspace_bytes(int32_t side);
size_t dg_tv_workspace_bytes(int64_t n_pixels);
/* Work bytes of DG_DEN_TVW for an I x I image (0 for side <= 0). */
size_t dg_tvw_workspace_bytes(int32_t side);
dg_status denoise(const dg_plan* plan, int32_t kind, const void* params, const float* r,
                  const double* tau_r, uint64_t probe_seed, int32_t iter, double eps_rel,
                  float* x_out, double* div_out, void* work, void* stream);

/* Learned residual CNN denoiser D(r) = r - f(r) (a plug-in for the black-box
 * denoiser of Sec. 4.3): f = conv 1->64, ReLU, 8 x (conv 64->64, ReLU),
 * conv 64->1, all 3x3 with bias and zero padding; BF16 weights and
 * activations, FP32 accumulation (MFMA).  With DG_DEN_CNN the divergence of
 * eq. MC_SURE is taken in its eps -> 0 limit, b^T J_D(r) b / N, by a
 * forward-mode tangent pass through the ReLU pattern of r.
 * Master parameters: FP32, dg_cnn_param_count() values, per layer
 * w[co][ci][3][3] then b[co] (layers in order).  dg_cnn_pack converts them to
 * the packed device format (BF16 weights) that denoise and training use.   */
size_t dg_cnn_weight_bytes(void);
int64_t dg_cnn_param_count(void);
size_t dg_cnn_workspace_bytes(int64_t n_pixels);
dg_status dg_cnn_pack(const float* master, void* packed, void* stream);
/* out = D(in) for n images of h x w (FP32, row-major, back to back).        */
dg_status dg_cnn_forward(const void* packed, int32_t n, int32_t h, int32_t w, const float* in,
                         float* out, void* work, void* stream);
/* One Adam step (lr, betas 0.9/0.999, eps 1e-8, bias-corrected with `step`
 * >= 1) on L = mean((D(noisy) - clean)^2) over n images of h x w: forward,
 * backward (BF16 MFMA, FP32 accumulation), gradient into `grad`, Adam update
 * of `master` with moments adam_m/adam_v, repack into `packed`; *loss_out
 * (device double) receives L.  work: dg_cnn_workspace_bytes(n*h*w).        */
dg_status dg_cnn_train_step(const float* noisy, const float* clean, int32_t n, int32_t h,
                            int32_t w, float* master, void* packed, float* grad, float* adam_m,
                            float* adam_v, int32_t step, double lr, double* loss_out, void* work,
                            void* stream);

/* D-GAMP-CT iterations (Algorithm 1, Sec. 4), with Phi~ = A V^-1:
 *   z = Phi~ x; tau_p = fro2 tau_x / M; p = z - tau_p s_prev;
 *   (s, tau_s) = channel(p, y, tau_p); tau_r = N / (fro2 tau_s);
 *   r = x + tau_r Phi~^T s; x = D(r); tau_x = tau_r div
 * optionally damped (Sec. 7): from the second iteration on, (s, tau_s) and
 * (x, tau_x) are mixed with their previous values by eta_s and eta_x.
 * A non-positive divergence sets tau_x = 1e-12 tau_r (counted in the log).
 * state: x (N), s (M) device floats; scal: device doubles, DG_NSCAL of them
 * (tau_x, tau_p, tau_s, tau_r, div, eps, status, clamps); state->t counts
 * the iterations done (host).  mu_out (nullable): V^-1 x after the last
 * iteration.  log (nullable, device): n_iter * DG_LOG_STRIDE doubles
 * (tau_p, tau_s, tau_r, div, tau_x, eps, status).
 * A non-finite or non-positive variance sets scal[DG_S_STATUS] to 1 + the
 * failing iteration; later iterations leave the state unchanged.           */
#define DG_NSCAL 16
#define DG_S_TAU_X 0
#define DG_S_TAU_P 1
#define DG_S_TAU_S 2
#define DG_S_TAU_R 3
#define DG_S_DIV 4
#define DG_S_EPS 5
#define DG_S_STATUS 6
#define DG_S_CLAMPS 7
#define DG_LOG_STRIDE 8
typedef struct dgamp_opts {
  int32_t n_iter;
  int32_t den_kind;
  const void* den_params;  /* host pointer, struct matching den_kind          */
  double fro2;             /* ||A V^-1||_F^2                                  */
  double i0;               /* source intensity (photons per ray)             */
  uint64_t probe_seed;
  double eps_rel;          /* MC step relative to max|r| (1e-3)               */
  double eta_x, eta_s;     /* damping, 1 = Algorithm 1 verbatim               */
  int32_t onsager;         /* 0: p = z (no Onsager term)                      */
  int32_t channel_mode;    /* DG_CHANNEL_*                                    */
  void** phase_events;     /* NULL, or a host array of n_iter*(DG_NPHASES+1)
                              hipEvent_t recorded on `stream` before the first
                              and after each phase of every iteration:
                              V^-1 x | A | channel | A^T | V^-1 g + r update |
                              denoiser | divergence + tau_x                   */
  uint32_t phase_mask;     /* 0: record every mark; else only the marks k
                              (0..DG_NPHASES) with bit k set (fewer event
                              records inside a timed run)                     */
} dgamp_opts;
#define DG_NPHASES 7
typedef struct dgamp_state {
  float* x;      /* device, N: x^t                     */
  float* s;      /* device, M: s^{t-1}                 */
  double* scal;  /* device, DG_NSCAL                   */
  int32_t t;     /* host: iterations already done      */
} dgamp_state;

/* x = 0, s = 0, tau_x = tau_x0, all other scalars 0, t = 0.                 */
dg_status dgamp_state_init(const dg_plan* plan, dgamp_state* st, double tau_x0, void* stream);
dg_status dgamp_iterate(const dg_plan* plan, const float* y, const dgamp_opts* opts,
                        dgamp_state* st, float* mu_out, double* log, void* work,
                        void* stream);

/* Synchronous status check of the asynchronous iteration calls (Algorithm 1
 * stops being meaningful once a variance tau is non-finite or <= 0).
 * Synchronises `stream`, reads the status word of n_slices consecutive
 * scalar blocks (scal: device, n_slices * DG_NSCAL doubles, as dgamp_state
 * or a batch holds them) and returns DG_ERR_NUMERIC for the first slice whose
 * status is set, with that slice and its failing iteration in *failed_slice
 * and *failed_iter (both nullable; -1 when every slice is fine) and in
 * dg_last_error(); DG_OK otherwise.                                          */
dg_status dg_check_status(const double* scal, int32_t n_slices, int32_t* failed_slice,
                          int32_t* failed_iter, void* stream);

/* dgamp_iterate without a workspace argument and without any device
 * allocation, for callers that cannot allocate (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, kernels
 * and results as dgamp_iterate; the iteration workspace is a fixed device
 * array inside the library, dg_noalloc_scratch_bytes() = 48 MiB on every
 * GPU the library runs on, held until the process ends.  A plan whose
 * dg_workspace_bytes(plan, DG_OP_DGAMP) exceeds it returns DG_ERR_ARG with
 * nothing launched (every image side up to 1024 with up to ~10^6 rays fits).
 * The first call on a device looks up the array's device address (no
 * allocation).  All calls on one GPU share the array: calls that overlap on
 * one GPU (different streams or threads) race.  Buffers a denoiser takes
 * through den_params (CNN activations, the TV kinds' state) stay the
 * caller's, as with dgamp_iterate.                                          */
size_t dg_noalloc_scratch_bytes(void);
dg_status dgamp_iterate_noalloc(const dg_plan* plan, const float* y, const dgamp_opts* opts,
                                dgamp_state* st, float* mu_out, double* log, void* stream);

/* Scalar state evolution of D-GAMP-CT (Sec. 4.4, eqs. SEasym and SE_matches;
 * the error function E_in and the sensitivity function A_in), evaluated on a
 * known phantom with the iteration's own channel and denoiser kernels.  For
 * t = 0 .. opts->n_iter - 1, from tau_x = tau_x0:
 *   tau_p = fro2 tau_x / M;  P = z + sqrt(tau_p) n;
 *   tau_s = sum_i (1 - Var[z_i | P_i, y_i, tau_p] / tau_p) / (M tau_p)
 *           (-E[d g_out / dp] of the matched channel), damped by eta_s from t = 1;
 *   tau_r = N / (fro2 tau_s) = xi_r;  R = x + sqrt(tau_r) v;
 *   D(R) and div (one probe, eq. MC_SURE, iteration index t);
 *   E_in = ||D(R) - x||^2 / N  (the predicted MSE of the denoiser's output);
 *   tau_x = tau_r div (A_in; div <= 0 gives 1e-12 tau_r), damped by eta_x.
 * z: M floats, the true line integrals A mu; x: N floats, V mu (the
 * preconditioned-domain signal); y: M counts; n: M and v: N floats, standard
 * normal fields supplied by the caller (all device).  Denoiser, i0, fro2,
 * probe seed, eps_rel, damping and channel mode from opts (phase_events must
 * be NULL; onsager is unused).  se_log (device, nullable): n_iter *
 * DG_LOG_STRIDE doubles per iteration (tau_p, tau_s, tau_r, div, tau_x,
 * E_in at DG_SE_LOG_MSE, status, clamps).  scal_out (device, nullable):
 * the final DG_NSCAL scalars.  A non-finite or non-positive variance sets
 * the status word to 1 + t and freezes the scalars.
 * work: dg_workspace_bytes(plan, DG_OP_SE).                                 */
#define DG_SE_LOG_MSE 5
dg_status dgamp_state_evolution(const dg_plan* plan, const float* z, const float* x,
                                const float* y, const float* n, const float* v,
                                const dgamp_opts* opts, double tau_x0, double* se_log,
                                double* scal_out, void* work, void* stream);

/* A whole reconstruction as one replayable HIP graph: optional state reset
 * (dgamp_state_init with tau_x0 when tau_x0 > 0), then opts->n_iter
 * iterations of dgamp_iterate and the final mu_out = V^-1 x, captured once
 * and instantiated.  Every dg_graph_launch replays exactly that sequence
 * (the same iteration indices, hence the same probes) on `stream`; the
 * buffers named at creation must stay valid while the graph exists.
 * opts->phase_events must be NULL.  Capture uses a private stream, so the
 * caller's stream may be the legacy default stream.                        */
typedef struct dg_graph dg_graph;
dg_status dgamp_graph_create(const dg_plan* plan, const float* y, const dgamp_opts* opts,
                             dgamp_state* st, double tau_x0, float* mu_out, double* log,
                             void* work, dg_graph** out);
dg_status dg_graph_launch(dg_graph* g, void* stream);
dg_status dg_graph_destroy(dg_graph* g);

/* ||A V^-1||_F^2 by Hutchinson's estimator over n_probes Rademacher probes
 * b_k (b_k,i = 1 - 2 (SplitMix64(seed ^ (k << 32) ^ i) & 1)):
 * mean_k ||A V^-1 b_k||^2, FP64 accumulation; written to *out (device).
 * work: dg_workspace_bytes(DG_OP_FRO2).                                     */
dg_status dg_fro2_hutchinson(const dg_plan* plan, int32_t n_probes, uint64_t seed,
                             double* out, void* work, void* stream);

/* Reconstruction PSNR as Sec. 6 reports it: 10 log10(peak^2 / MSE), peak =
 * max(0, max_i ref_i) (attenuation images are non-negative), MSE over all n
 * pixels, FP64 accumulation; written to *out (device double).  est, ref:
 * device FP32, n >= 1; work: dg_psnr_workspace_bytes() device bytes.  A zero
 * MSE gives +inf, non-finite input NaN.                                     */
size_t dg_psnr_workspace_bytes(void);
dg_status dg_psnr(int64_t n, const float* est, const float* ref, double* out, void* work,
                  void* stream);

/* ------------------------------------------------------------------ batch
 * Many independent slices in one set of launches (not in the paper, whose
 * method reconstructs one slice at a time; every slice runs exactly the
 * iteration of Algorithm 1 that dgamp_iterate runs, with its own scalars).
 * Slices may differ in image side and view count; each phase of an
 * iteration (V^-1, A, channel, A^T, V^-1 + r update, denoiser, divergence)
 * is one launch over the blocks of every slice.  Small slices that would
 * leave most compute units idle on their own fill the chip together.
 *
 * Layout: the batch's images and sinograms are packed back to back; slice k
 * owns x[img_off[k] .. img_off[k+1]) (row-major I_k x I_k) and
 * y, s[sino_off[k] .. sino_off[k+1]) (view-major), and scal[k*DG_NSCAL ..].
 * All buffers are device memory owned by the caller.                        */
typedef struct dg_batch dg_batch;

/* Build one plan per distinct geometry (n in 1..4096, every image side
 * supported by the preconditioner FFT, else DG_ERR_UNSUPPORTED); slices
 * with equal dg_geom fields share a plan and its device tables.            */
dg_status dg_batch_create(const dg_geom* geoms, int32_t n, dg_batch** out);
dg_status dg_batch_destroy(dg_batch* b);
/* Host arrays of n+1 entries: element offsets of every slice's image and
 * sinogram (the last entry is the total).                                   */
dg_status dg_batch_layout(const dg_batch* b, int64_t* img_off, int64_t* sino_off);
/* Bytes of the work buffer dg_batch_bind takes (256-byte aligned device).  */
size_t dg_batch_workspace_bytes(const dg_batch* b);
/* Bind the batch to its buffers and build the per-slice argument tables
 * (device uploads; call outside any stream capture).  y: counts; i0, fro2:
 * host arrays of n (source intensity and ||A V^-1||_F^2 per slice); x, s,
 * scal: the state (as dgamp_state, packed); mu_out: NULL, or where
 * mu = V^-1 x lands when an iteration call asks for it.  den_kind is
 * DG_DEN_NLM (dg_nlm_params) or DG_DEN_CNN (dg_cnn_params; all slices of
 * one side, its work buffer sized for dg_cnn_workspace_bytes(totN));
 * DG_DEN_HAAR is DG_ERR_UNSUPPORTED here.  den_params is copied.           */
dg_status dg_batch_bind(dg_batch* b, const float* y, const double* i0, const double* fro2,
                        float* x, float* s, double* scal, float* mu_out, int32_t den_kind,
                        const void* den_params, double eps_rel, void* work);
/* Every slice's state as dgamp_state_init sets it.                          */
dg_status dg_batch_state_init(dg_batch* b, double tau_x0, void* stream);
/* n_iter iterations t0 .. t0+n_iter-1 of every slice, then mu_out when
 * write_mu != 0.  Arguments as the fields of dgamp_opts.  Slice k's result
 * equals that of dgamp_iterate on its own plan with the same arguments.     */
dg_status dgamp_batch_iterate(dg_batch* b, int32_t n_iter, int32_t t0, uint64_t probe_seed,
                              double eta_x, double eta_s, int32_t onsager,
                              int32_t channel_mode, int32_t write_mu, void* stream);
/* dg_batch_state_init + dgamp_batch_iterate(t0 = 0, write_mu when mu_out
 * was bound) captured as one graph, replayed by dg_graph_launch.            */
dg_status dg_batch_graph_create(dg_batch* b, double tau_x0, int32_t n_iter,
                                uint64_t probe_seed, double eta_x, double eta_s,
                                int32_t onsager, int32_t channel_mode, dg_graph** out);

/* ------------------------------------------------------------------ autotune
 * The forward projector splits every ray's march into 2, 4, 8 or 16 segments
 * handled by different lanes (variants 0, 1, 2, 3; default 1).  The variants
 * sum the same chord-weighted pixels in a different order, so sinograms
 * agree to FP32 rounding (relative ~1e-7), not bit for bit.  The autotune
 * calls time each variant `reps` times on the given data (synchronising the
 * stream) and keep the fastest for later calls on the plan or batch; the
 * batch tuner overwrites the batch's z work buffer only, the plan tuner
 * writes `sino` (img_t may be NULL).  The setters restore a stored choice
 * (variant outside 0..3: DG_ERR_ARG).                                       */
dg_status dg_batch_autotune(dg_batch* b, int32_t reps, void* stream);
int32_t dg_batch_projector_variant(const dg_batch* b);
dg_status dg_batch_set_projector_variant(dg_batch* b, int32_t variant);
dg_status dg_plan_autotune(dg_plan* plan, const float* img, const float* img_t, float* sino,
                           int32_t reps, void* stream);
int32_t dg_plan_projector_variant(const dg_plan* plan);
dg_status dg_plan_set_projector_variant(dg_plan* plan, int32_t variant);

/* The non-local-means denoiser splits a 32 x 32 tile's search offsets over
 * 8 or 4 wavefronts (variants 0, 1; default 0): a tile of 4 wavefronts
 * needs half the LDS, so two share a compute unit, while 8 fill more
 * compute units when an image has few tiles.  The variants add the
 * offsets' partial sums in different groupings, so outputs agree to FP32
 * rounding, not bit for bit.  dg_plan_autotune_nlm times both `reps` times
 * on r (N floats) with fixed tau_r and eps, writing out (2N floats,
 * D(r) then D(r + eps b)); it allocates a 16-byte scratch pair and
 * synchronises the stream.  dg_batch_autotune also times them on the bound
 * batch when its denoiser is non-local means (outputs into the batch's
 * work buffers; the iteration state is not touched).  The setters restore
 * a stored choice (variant outside 0..1: DG_ERR_ARG).                       */
dg_status dg_plan_autotune_nlm(dg_plan* plan, const dg_nlm_params* params, const float* r,
                               float* out, int32_t reps, void* stream);
int32_t dg_plan_nlm_variant(const dg_plan* plan);
dg_status dg_plan_set_nlm_variant(dg_plan* plan, int32_t variant);
int32_t dg_batch_nlm_variant(const dg_batch* b);
dg_status dg_batch_set_nlm_variant(dg_batch* b, int32_t variant);

#ifdef __cplusplus
}
#endif
#endif /* DGAMPCT_H */
