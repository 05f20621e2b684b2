"""Python binding of libdgampct.so: argument marshalling only.

Each function has the name of the C entry point it calls (see
include/dgampct.h).  Tensors must be contiguous CUDA (HIP) tensors of the
stated dtype; calls are enqueued on torch's current stream.  Nothing here
computes any part of the method: a missing or unloadable library raises
instead of falling back.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgampct.so")

PARALLEL, FAN = 0, 1
DEN_HAAR, DEN_NLM, DEN_CNN, DEN_TV, DEN_TVW, DEN_BM3D = 0, 1, 2, 3, 4, 5
CHANNEL_LAPLACE, CHANNEL_MODE_ONLY = 0, 1
OP_PRECOND, OP_DENOISE, OP_DGAMP, OP_FRO2, OP_SE = 0, 1, 2, 3, 4
SE_LOG_MSE = 5
ERR_ARG, ERR_HIP, ERR_NUMERIC, ERR_UNSUPPORTED, ERR_NOMEM = -1, -2, -3, -4, -5
NSCAL = 16
S_TAU_X, S_TAU_P, S_TAU_S, S_TAU_R, S_DIV, S_EPS, S_STATUS, S_CLAMPS = range(8)
LOG_STRIDE = 8
LOG_FIELDS = ("tau_p", "tau_s", "tau_r", "div", "tau_x", "eps", "status", "clamps")
# column of each field in a per-iteration log record (not the scalar-block indices S_*)
LOG_TAU_P, LOG_TAU_S, LOG_TAU_R, LOG_DIV, LOG_TAU_X, LOG_EPS, LOG_STATUS = range(7)
NPHASES = 7
PHASES = ("precond_x", "project", "channel", "backproject", "precond_g_update", "denoise", "div")

EXPORTS = ("dg_plan_create", "dg_plan_destroy", "dg_workspace_bytes", "dg_channel_workspace_bytes",
           "dg_last_error", "ct_project", "ct_backproject", "ct_precondition", "gamp_poisson_out",
           "denoise", "dgamp_state_init", "dgamp_iterate", "dg_fro2_hutchinson",
           "dgamp_graph_create", "dg_graph_launch", "dg_graph_destroy", "dg_cnn_weight_bytes",
           "dg_cnn_param_count", "dg_cnn_workspace_bytes", "dg_cnn_pack", "dg_cnn_forward",
           "dg_cnn_train_step", "dg_batch_create", "dg_batch_destroy", "dg_batch_layout",
           "dg_batch_workspace_bytes", "dg_batch_bind", "dg_batch_state_init",
           "dgamp_batch_iterate", "dg_batch_graph_create", "dg_batch_autotune",
           "dg_batch_projector_variant", "dg_plan_autotune", "dg_plan_projector_variant",
           "dg_batch_set_projector_variant", "dg_plan_set_projector_variant",
           "dg_psnr_workspace_bytes", "dg_psnr", "dg_tv_workspace_bytes", "dg_tvw_workspace_bytes",
           "dg_check_status", "dg_noalloc_scratch_bytes", "dgamp_iterate_noalloc",
           "dgamp_state_evolution", "dg_bm3d_workspace_bytes", "dg_fourier_create", "dg_fourier_destroy",
           "dg_fourier_workspace_bytes", "ct_project_fourier", "ct_backproject_fourier",
           "dg_plan_autotune_nlm", "dg_plan_nlm_variant", "dg_plan_set_nlm_variant",
           "dg_batch_nlm_variant", "dg_batch_set_nlm_variant")


class DgError(RuntimeError):
    pass


class Geom(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("n_views", ctypes.c_int32),
                ("n_bins", ctypes.c_int32), ("pixel_mm", ctypes.c_double),
                ("angle0_rad", ctypes.c_double), ("span_rad", ctypes.c_double),
                ("bin_mm", ctypes.c_double), ("dso_mm", ctypes.c_double),
                ("ddo_mm", ctypes.c_double), ("dgamma_rad", ctypes.c_double)]


class HaarParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("levels", ctypes.c_int32)]


class NlmParams(ctypes.Structure):
    _fields_ = [("patch_radius", ctypes.c_int32), ("search_radius", ctypes.c_int32),
                ("hfac", ctypes.c_double)]


class CnnParams(ctypes.Structure):
    _fields_ = [("weights", ctypes.c_void_p), ("work", ctypes.c_void_p)]


class TvParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("iters", ctypes.c_int32), ("metric", ctypes.c_int32),
                ("work", ctypes.c_void_p)]


class Bm3dParams(ctypes.Structure):
    _fields_ = [("work", ctypes.c_void_p)]


class DgampOpts(ctypes.Structure):
    _fields_ = [("n_iter", ctypes.c_int32), ("den_kind", ctypes.c_int32),
                ("den_params", ctypes.c_void_p), ("fro2", ctypes.c_double), ("i0", ctypes.c_double),
                ("probe_seed", ctypes.c_uint64), ("eps_rel", ctypes.c_double),
                ("eta_x", ctypes.c_double), ("eta_s", ctypes.c_double),
                ("onsager", ctypes.c_int32), ("channel_mode", ctypes.c_int32),
                ("phase_events", ctypes.c_void_p), ("phase_mask", ctypes.c_uint32)]


class DgampStateC(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("s", ctypes.c_void_p), ("scal", ctypes.c_void_p),
                ("t", ctypes.c_int32)]


_lib = None
_VP = ctypes.c_void_p


def load():
    """Load the HIP library (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise DgError("libdgampct.so is not built (run paper_1609_04661_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, u64, dbl, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "dg_plan_create": ([ctypes.POINTER(Geom), ctypes.POINTER(_VP)], i32),
        "dg_plan_destroy": ([_VP], i32),
        "dg_workspace_bytes": ([_VP, i32], sz),
        "dg_channel_workspace_bytes": ([i64], sz),
        "dg_last_error": ([], ctypes.c_char_p),
        "ct_project": ([_VP, _VP, _VP, _VP, _VP], i32),
        "ct_backproject": ([_VP, _VP, _VP, _VP], i32),
        "ct_precondition": ([_VP, i32, _VP, _VP, _VP, _VP], i32),
        "gamp_poisson_out": ([i64, _VP, _VP, _VP, dbl, i32, _VP, _VP, _VP, _VP], i32),
        "denoise": ([_VP, i32, _VP, _VP, _VP, u64, i32, dbl, _VP, _VP, _VP, _VP], i32),
        "dgamp_state_init": ([_VP, ctypes.POINTER(DgampStateC), dbl, _VP], i32),
        "dgamp_iterate": ([_VP, _VP, ctypes.POINTER(DgampOpts), ctypes.POINTER(DgampStateC), _VP,
                           _VP, _VP, _VP], i32),
        "dg_fro2_hutchinson": ([_VP, i32, u64, _VP, _VP, _VP], i32),
        "dgamp_graph_create": ([_VP, _VP, ctypes.POINTER(DgampOpts), ctypes.POINTER(DgampStateC),
                                dbl, _VP, _VP, _VP, ctypes.POINTER(_VP)], i32),
        "dg_graph_launch": ([_VP, _VP], i32),
        "dg_graph_destroy": ([_VP], i32),
        "dg_cnn_weight_bytes": ([], sz),
        "dg_cnn_param_count": ([], i64),
        "dg_cnn_workspace_bytes": ([i64], sz),
        "dg_cnn_pack": ([_VP, _VP, _VP], i32),
        "dg_cnn_forward": ([_VP, i32, i32, i32, _VP, _VP, _VP, _VP], i32),
        "dg_cnn_train_step": ([_VP, _VP, i32, i32, i32, _VP, _VP, _VP, _VP, _VP, i32, dbl, _VP,
                               _VP, _VP], i32),
        "dg_batch_create": ([ctypes.POINTER(Geom), i32, ctypes.POINTER(_VP)], i32),
        "dg_batch_destroy": ([_VP], i32),
        "dg_batch_layout": ([_VP, ctypes.POINTER(i64), ctypes.POINTER(i64)], i32),
        "dg_batch_workspace_bytes": ([_VP], sz),
        "dg_batch_bind": ([_VP, _VP, ctypes.POINTER(dbl), ctypes.POINTER(dbl), _VP, _VP, _VP, _VP,
                           i32, _VP, dbl, _VP], i32),
        "dg_batch_state_init": ([_VP, dbl, _VP], i32),
        "dgamp_batch_iterate": ([_VP, i32, i32, u64, dbl, dbl, i32, i32, i32, _VP], i32),
        "dg_batch_graph_create": ([_VP, dbl, i32, u64, dbl, dbl, i32, i32, ctypes.POINTER(_VP)],
                                  i32),
        "dg_batch_autotune": ([_VP, i32, _VP], i32),
        "dg_batch_projector_variant": ([_VP], i32),
        "dg_plan_autotune": ([_VP, _VP, _VP, _VP, i32, _VP], i32),
        "dg_plan_projector_variant": ([_VP], i32),
        "dg_batch_set_projector_variant": ([_VP, i32], i32),
        "dg_plan_set_projector_variant": ([_VP, i32], i32),
        "dg_plan_autotune_nlm": ([_VP, _VP, _VP, _VP, i32, _VP], i32),
        "dg_plan_nlm_variant": ([_VP], i32),
        "dg_plan_set_nlm_variant": ([_VP, i32], i32),
        "dg_batch_nlm_variant": ([_VP], i32),
        "dg_batch_set_nlm_variant": ([_VP, i32], i32),
        "dg_psnr_workspace_bytes": ([], sz),
        "dg_psnr": ([i64, _VP, _VP, _VP, _VP, _VP], i32),
        "dg_tv_workspace_bytes": ([i64], sz),
        "dg_tvw_workspace_bytes": ([i32], sz),
        "dg_check_status": ([_VP, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), _VP], i32),
        "dg_noalloc_scratch_bytes": ([], sz),
        "dg_bm3d_workspace_bytes": ([i32], sz),
        "dg_fourier_create": ([ctypes.POINTER(Geom), ctypes.POINTER(_VP)], i32),
        "dg_fourier_destroy": ([_VP], i32),
        "dg_fourier_workspace_bytes": ([_VP], sz),
        "ct_project_fourier": ([_VP, _VP, _VP, _VP, _VP], i32),
        "ct_backproject_fourier": ([_VP, _VP, _VP, _VP, _VP], i32),
        "dgamp_state_evolution": ([_VP, _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(DgampOpts), dbl,
                                   _VP, _VP, _VP, _VP], i32),
        "dgamp_iterate_noalloc": ([_VP, _VP, ctypes.POINTER(DgampOpts), ctypes.POINTER(DgampStateC),
                                   _VP, _VP, _VP], i32),
    }
    missing = set(EXPORTS) - set(sig)
    if missing:
        raise DgError("no ctypes signature for %s" % sorted(missing))
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        msg = _lib.dg_last_error().decode(errors="replace")
        raise DgError("status %d: %s" % (rc, msg))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise DgError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise DgError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise DgError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise DgError("%s must have %d elements, got %d" % (name, numel, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A dg_plan for one geometry (dict with the dg_geom fields)."""

    def __init__(self, geom):
        L = load()
        self.geom = dict(geom)
        g = Geom(**{k: self.geom[k] for k, _ in Geom._fields_})
        h = _VP()
        _check(L.dg_plan_create(ctypes.byref(g), ctypes.byref(h)))
        self._h = h
        self.I = int(geom["n"])
        self.N = self.I * self.I
        self.M = int(geom["n_views"]) * int(geom["n_bins"])
        self.shape_sino = (int(geom["n_views"]), int(geom["n_bins"]))

    @property
    def handle(self):
        return self._h

    def workspace(self, op):
        n = int(_lib.dg_workspace_bytes(self._h, op))
        return torch.empty(max(n, 256), dtype=torch.uint8, device="cuda")

    def autotune(self, img, img_t=None, sino=None, reps=10):
        """Time the projector variants on `img` and keep the fastest."""
        if sino is None:
            sino = torch.empty(self.shape_sino, dtype=torch.float32, device="cuda")
        _check(_lib.dg_plan_autotune(self._h, _ptr(img, torch.float32, self.N, "img"),
                                     _ptr(img_t, torch.float32, self.N, "img_t"),
                                     _ptr(sino, torch.float32, self.M, "sino"), int(reps),
                                     _stream()))
        return int(_lib.dg_plan_projector_variant(self._h))

    @property
    def projector_variant(self):
        return int(_lib.dg_plan_projector_variant(self._h))

    @projector_variant.setter
    def projector_variant(self, v):
        _check(_lib.dg_plan_set_projector_variant(self._h, int(v)))

    def autotune_nlm(self, r, params=None, reps=10):
        """Time the non-local-means variants on `r` and keep the faster."""
        if params is None:
            params = make_params(DEN_NLM)
        out = torch.empty(2 * self.N, dtype=torch.float32, device="cuda")
        _check(_lib.dg_plan_autotune_nlm(self._h, ctypes.byref(params),
                                         _ptr(r, torch.float32, self.N, "r"),
                                         _ptr(out, torch.float32, 2 * self.N, "out"), int(reps),
                                         _stream()))
        return int(_lib.dg_plan_nlm_variant(self._h))

    @property
    def nlm_variant(self):
        return int(_lib.dg_plan_nlm_variant(self._h))

    @nlm_variant.setter
    def nlm_variant(self, v):
        _check(_lib.dg_plan_set_nlm_variant(self._h, int(v)))

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _lib is not None:
                _lib.dg_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass


def ct_project(plan, img, img_t=None, sino=None):
    if sino is None:
        sino = torch.empty(plan.shape_sino, dtype=torch.float32, device="cuda")
    _check(_lib.ct_project(plan.handle, _ptr(img, torch.float32, plan.N, "img"),
                           _ptr(img_t, torch.float32, plan.N, "img_t"),
                           _ptr(sino, torch.float32, plan.M, "sino"), _stream()))
    return sino


def ct_backproject(plan, sino, img=None):
    if img is None:
        img = torch.empty((plan.I, plan.I), dtype=torch.float32, device="cuda")
    _check(_lib.ct_backproject(plan.handle, _ptr(sino, torch.float32, plan.M, "sino"),
                               _ptr(img, torch.float32, plan.N, "img"), _stream()))
    return img


def ct_precondition(plan, direction, inp, out=None, work=None):
    if out is None:
        out = torch.empty((plan.I, plan.I), dtype=torch.float32, device="cuda")
    if work is None:
        work = plan.workspace(OP_PRECOND)
    _check(_lib.ct_precondition(plan.handle, int(direction), _ptr(inp, torch.float32, plan.N, "in"),
                                _ptr(out, torch.float32, plan.N, "out"),
                                _ptr(work, torch.uint8, None, "work"), _stream()))
    return out


def gamp_poisson_out(p, y, tau_p, i0, mode=CHANNEL_LAPLACE, s_out=None, tau_s_out=None, work=None):
    m = p.numel()
    if s_out is None:
        s_out = torch.empty_like(p)
    if tau_s_out is None:
        tau_s_out = torch.empty(1, dtype=torch.float64, device="cuda")
    if work is None:
        work = torch.empty(int(_lib.dg_channel_workspace_bytes(m)), dtype=torch.uint8, device="cuda")
    _check(_lib.gamp_poisson_out(m, _ptr(p, torch.float32, m, "p"), _ptr(y, torch.float32, m, "y"),
                                 _ptr(tau_p, torch.float64, 1, "tau_p"), float(i0), int(mode),
                                 _ptr(s_out, torch.float32, m, "s_out"),
                                 _ptr(tau_s_out, torch.float64, 1, "tau_s_out"),
                                 _ptr(work, torch.uint8, None, "work"), _stream()))
    return s_out, tau_s_out


def make_params(kind, **kw):
    if kind == DEN_HAAR:
        return HaarParams(alpha=kw.get("alpha", 1.5), levels=kw.get("levels", 0))
    if kind == DEN_NLM:
        return NlmParams(patch_radius=kw.get("pr", 2), search_radius=kw.get("sr", 10),
                         hfac=kw.get("hfac", 0.4))
    if kind == DEN_CNN:
        net = kw["net"]
        return CnnParams(weights=ctypes.c_void_p(net.packed.data_ptr()),
                         work=ctypes.c_void_p(net.work_for(kw["n_pixels"]).data_ptr()))
    if kind == DEN_TV:
        # the dual-state buffer lives as long as the params object
        buf = torch.empty(int(load().dg_tv_workspace_bytes(int(kw["n_pixels"]))), dtype=torch.uint8,
                          device="cuda")
        prm = TvParams(alpha=kw.get("alpha", 0.5), iters=kw.get("iters", 50),
                       work=ctypes.c_void_p(buf.data_ptr()))
        prm._buf = buf
        return prm
    if kind == DEN_TVW:
        # the solver state (primal, dual, spectra) lives as long as the params object
        buf = torch.empty(int(load().dg_tvw_workspace_bytes(int(kw["side"]))), dtype=torch.uint8,
                          device="cuda")
        prm = TvParams(alpha=kw.get("alpha", 1.0), iters=kw.get("iters", 50),
                       metric=kw.get("metric", 0), work=ctypes.c_void_p(buf.data_ptr()))
        prm._buf = buf
        return prm
    if kind == DEN_BM3D:
        # groups, accumulators and the basic estimate live as long as the params object
        buf = torch.empty(max(int(load().dg_bm3d_workspace_bytes(int(kw["side"]))), 256),
                          dtype=torch.uint8, device="cuda")
        prm = Bm3dParams(work=ctypes.c_void_p(buf.data_ptr()))
        prm._buf = buf
        return prm
    raise DgError("unknown denoiser kind")


def denoise(plan, kind, params, r, tau_r, probe_seed=0, iteration=0, eps_rel=1e-3, x_out=None,
            div_out=None, with_div=True, work=None):
    if x_out is None:
        x_out = torch.empty((plan.I, plan.I), dtype=torch.float32, device="cuda")
    if with_div and div_out is None:
        div_out = torch.empty(1, dtype=torch.float64, device="cuda")
    if work is None:
        work = plan.workspace(OP_DENOISE)
    _check(_lib.denoise(plan.handle, int(kind), ctypes.byref(params),
                        _ptr(r, torch.float32, plan.N, "r"), _ptr(tau_r, torch.float64, 1, "tau_r"),
                        int(probe_seed), int(iteration), float(eps_rel),
                        _ptr(x_out, torch.float32, plan.N, "x_out"),
                        _ptr(div_out, torch.float64, 1, "div_out") if with_div else None,
                        _ptr(work, torch.uint8, None, "work"), _stream()))
    return x_out, div_out


class DgampState:
    """Device state of a D-GAMP-CT run: x^t, s^{t-1} and the scalar block."""

    def __init__(self, plan, tau_x0=1.0):
        self.plan = plan
        self.x = torch.zeros((plan.I, plan.I), dtype=torch.float32, device="cuda")
        self.s = torch.zeros(plan.shape_sino, dtype=torch.float32, device="cuda")
        self.scal = torch.zeros(NSCAL, dtype=torch.float64, device="cuda")
        self.c = DgampStateC(x=self.x.data_ptr(), s=self.s.data_ptr(), scal=self.scal.data_ptr(), t=0)
        _check(_lib.dgamp_state_init(plan.handle, ctypes.byref(self.c), float(tau_x0), _stream()))

    @property
    def t(self):
        return self.c.t


def make_opts(n_iter, fro2, i0, den_kind, den_params, probe_seed=0, eps_rel=1e-3, eta_x=1.0,
              eta_s=1.0, onsager=True, channel_mode=CHANNEL_LAPLACE, phase_events=None,
              phase_mask=0):
    return DgampOpts(n_iter=int(n_iter), den_kind=int(den_kind),
                     den_params=ctypes.cast(ctypes.pointer(den_params), ctypes.c_void_p),
                     fro2=float(fro2), i0=float(i0), probe_seed=int(probe_seed),
                     eps_rel=float(eps_rel), eta_x=float(eta_x), eta_s=float(eta_s),
                     onsager=1 if onsager else 0, channel_mode=int(channel_mode),
                     phase_events=ctypes.cast(phase_events, ctypes.c_void_p)
                     if phase_events is not None else None, phase_mask=int(phase_mask))


def dgamp_iterate(plan, y, state, n_iter, fro2, i0, den_kind, den_params, probe_seed=0,
                  eps_rel=1e-3, eta_x=1.0, eta_s=1.0, onsager=True, channel_mode=CHANNEL_LAPLACE,
                  mu_out=None, log=None, work=None, phase_events=None, phase_mask=0):
    """phase_events: optional ctypes array of n_iter * (NPHASES + 1) hipEvent_t handles;
    phase_mask: 0 records every mark, else only marks k with bit k set."""
    opts = make_opts(n_iter, fro2, i0, den_kind, den_params, probe_seed, eps_rel, eta_x, eta_s,
                     onsager, channel_mode, phase_events, phase_mask)
    if work is None:
        work = plan.workspace(OP_DGAMP)
    if log is not None and log.numel() < n_iter * LOG_STRIDE:
        raise DgError("log needs n_iter * %d doubles" % LOG_STRIDE)
    _check(_lib.dgamp_iterate(plan.handle, _ptr(y, torch.float32, plan.M, "y"), ctypes.byref(opts),
                              ctypes.byref(state.c), _ptr(mu_out, torch.float32, plan.N, "mu_out"),
                              _ptr(log, torch.float64, None, "log"),
                              _ptr(work, torch.uint8, None, "work"), _stream()))
    return mu_out


class FourierOp:
    """The Fourier-slice Radon operator of a parallel-beam geometry (device tables)."""

    def __init__(self, geom):
        g = Geom(**{k: geom[k] for k, _ in Geom._fields_})
        h = _VP()
        _check(_lib.dg_fourier_create(ctypes.byref(g), ctypes.byref(h)))
        self._h = h
        self.I, self.nv, self.nb = geom["n"], geom["n_views"], geom["n_bins"]
        self.work = torch.empty(max(int(_lib.dg_fourier_workspace_bytes(h)), 256), dtype=torch.uint8,
                                device="cuda")

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _lib is not None:
                _lib.dg_fourier_destroy(self._h)
                self._h = None
        except Exception:
            pass


def ct_project_fourier(op, img, sino=None):
    if sino is None:
        sino = torch.empty((op.nv, op.nb), dtype=torch.float32, device="cuda")
    _check(_lib.ct_project_fourier(op._h, _ptr(img, torch.float32, op.I * op.I, "img"),
                                   _ptr(sino, torch.float32, op.nv * op.nb, "sino"),
                                   _ptr(op.work, torch.uint8, None, "work"), _stream()))
    return sino


def ct_backproject_fourier(op, sino, img=None):
    if img is None:
        img = torch.empty((op.I, op.I), dtype=torch.float32, device="cuda")
    _check(_lib.ct_backproject_fourier(op._h, _ptr(sino, torch.float32, op.nv * op.nb, "sino"),
                                       _ptr(img, torch.float32, op.I * op.I, "img"),
                                       _ptr(op.work, torch.uint8, None, "work"), _stream()))
    return img


def dgamp_state_evolution(plan, z, x, y, n, v, n_iter, fro2, i0, den_kind, den_params,
                          probe_seed=0, eps_rel=1e-3, eta_x=1.0, eta_s=1.0,
                          channel_mode=CHANNEL_LAPLACE, tau_x0=1.0, log=None, scal_out=None,
                          work=None):
    """Scalar state evolution on a known phantom: z = A mu (M), x = V mu (N),
    y the counts, n (M) and v (N) standard-normal fields.  Returns the
    per-iteration log (n_iter x LOG_STRIDE, E_in at SE_LOG_MSE)."""
    opts = make_opts(n_iter, fro2, i0, den_kind, den_params, probe_seed, eps_rel, eta_x, eta_s,
                     True, channel_mode)
    if log is None:
        log = torch.zeros(max(n_iter, 1) * LOG_STRIDE, dtype=torch.float64, device="cuda")
    if work is None:
        work = plan.workspace(OP_SE)
    _check(_lib.dgamp_state_evolution(plan.handle, _ptr(z, torch.float32, plan.M, "z"),
                                      _ptr(x, torch.float32, plan.N, "x"),
                                      _ptr(y, torch.float32, plan.M, "y"),
                                      _ptr(n, torch.float32, plan.M, "n"),
                                      _ptr(v, torch.float32, plan.N, "v"), ctypes.byref(opts),
                                      float(tau_x0), _ptr(log, torch.float64, None, "log"),
                                      _ptr(scal_out, torch.float64, NSCAL, "scal_out"),
                                      _ptr(work, torch.uint8, None, "work"), _stream()))
    return log


def dgamp_iterate_noalloc(plan, y, state, n_iter, fro2, i0, den_kind, den_params, probe_seed=0,
                          eps_rel=1e-3, eta_x=1.0, eta_s=1.0, onsager=True,
                          channel_mode=CHANNEL_LAPLACE, mu_out=None, log=None):
    """dgamp_iterate with the library's fixed scratch array as its workspace."""
    opts = make_opts(n_iter, fro2, i0, den_kind, den_params, probe_seed, eps_rel, eta_x, eta_s,
                     onsager, channel_mode)
    if log is not None and log.numel() < n_iter * LOG_STRIDE:
        raise DgError("log needs n_iter * %d doubles" % LOG_STRIDE)
    _check(_lib.dgamp_iterate_noalloc(plan.handle, _ptr(y, torch.float32, plan.M, "y"),
                                      ctypes.byref(opts), ctypes.byref(state.c),
                                      _ptr(mu_out, torch.float32, plan.N, "mu_out"),
                                      _ptr(log, torch.float64, None, "log"), _stream()))
    return mu_out


def dg_noalloc_scratch_bytes():
    return int(_lib.dg_noalloc_scratch_bytes())


def dg_check_status(scal, n_slices=1):
    """Synchronise the current stream and read the status words: returns
    (status, failed_slice, failed_iter) with status 0 or ERR_NUMERIC (not
    raised), the indices -1 when every slice is fine."""
    fs, fi = ctypes.c_int32(), ctypes.c_int32()
    rc = _lib.dg_check_status(_ptr(scal, torch.float64, n_slices * NSCAL, "scal"), int(n_slices),
                              ctypes.byref(fs), ctypes.byref(fi), _stream())
    if rc not in (0, ERR_NUMERIC):
        _check(rc)
    return rc, fs.value, fi.value


def dg_fro2_hutchinson(plan, n_probes, seed, out=None, work=None):
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device="cuda")
    if work is None:
        work = plan.workspace(OP_FRO2)
    _check(_lib.dg_fro2_hutchinson(plan.handle, int(n_probes), int(seed),
                                   _ptr(out, torch.float64, 1, "out"),
                                   _ptr(work, torch.uint8, None, "work"), _stream()))
    return out


class DgampGraph:
    """A captured reconstruction (state reset + n_iter iterations + mu_out)."""

    def __init__(self, plan, y, state, n_iter, fro2, i0, den_kind, den_params, tau_x0=1.0,
                 mu_out=None, log=None, work=None, **kw):
        self.keep = (plan, y, state, den_params, mu_out, log)
        self.work = work if work is not None else plan.workspace(OP_DGAMP)
        self.opts = make_opts(n_iter, fro2, i0, den_kind, den_params, **kw)
        h = _VP()
        _check(_lib.dgamp_graph_create(plan.handle, _ptr(y, torch.float32, plan.M, "y"),
                                       ctypes.byref(self.opts), ctypes.byref(state.c),
                                       float(tau_x0), _ptr(mu_out, torch.float32, plan.N, "mu_out"),
                                       _ptr(log, torch.float64, None, "log"),
                                       _ptr(self.work, torch.uint8, None, "work"), ctypes.byref(h)))
        self._h = h

    def launch(self):
        _check(_lib.dg_graph_launch(self._h, _stream()))

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _lib is not None:
                _lib.dg_graph_destroy(self._h)
                self._h = None
        except Exception:
            pass


_psnr_work = {}


def dg_psnr(est, ref, out=None):
    """PSNR (dB) of est against ref on the device; returns a 1-element FP64 tensor."""
    n = ref.numel()
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device="cuda")
    dev = torch.cuda.current_device()
    if dev not in _psnr_work:
        _psnr_work[dev] = torch.empty(int(_lib.dg_psnr_workspace_bytes()), dtype=torch.uint8,
                                      device="cuda")
    _check(_lib.dg_psnr(n, _ptr(est, torch.float32, n, "est"), _ptr(ref, torch.float32, n, "ref"),
                        _ptr(out, torch.float64, 1, "out"),
                        _ptr(_psnr_work[dev], torch.uint8, None, "work"), _stream()))
    return out


class Batch:
    """Many slices (list of geometry dicts, image sides and view counts may
    differ) reconstructed together: images, sinograms and scalar blocks are
    packed back to back (``img_off``/``sino_off``); ``image(k)``/``sino(k)``
    give views of slice k."""

    def __init__(self, geoms):
        L = load()
        self.geoms = [dict(g) for g in geoms]
        n = len(self.geoms)
        arr = (Geom * n)(*[Geom(**{k: g[k] for k, _ in Geom._fields_}) for g in self.geoms])
        h = _VP()
        _check(L.dg_batch_create(arr, n, ctypes.byref(h)))
        self._h = h
        self.n = n
        io = (ctypes.c_int64 * (n + 1))()
        so = (ctypes.c_int64 * (n + 1))()
        _check(L.dg_batch_layout(h, io, so))
        self.img_off = [int(v) for v in io]
        self.sino_off = [int(v) for v in so]
        self.sides = [int(g["n"]) for g in self.geoms]
        self.sino_shapes = [(int(g["n_views"]), int(g["n_bins"])) for g in self.geoms]
        self.totN, self.totM = self.img_off[-1], self.sino_off[-1]
        self.x = torch.zeros(self.totN, dtype=torch.float32, device="cuda")
        self.s = torch.zeros(self.totM, dtype=torch.float32, device="cuda")
        self.scal = torch.zeros(n * NSCAL, dtype=torch.float64, device="cuda")
        self.work = torch.empty(max(int(L.dg_batch_workspace_bytes(h)), 256), dtype=torch.uint8,
                                device="cuda")
        self.keep = None

    def image(self, t, k):
        return t[self.img_off[k]:self.img_off[k + 1]].view(self.sides[k], self.sides[k])

    def sino(self, t, k):
        return t[self.sino_off[k]:self.sino_off[k + 1]].view(*self.sino_shapes[k])

    def bind(self, y, i0, fro2, den_kind, den_params, mu_out=None, eps_rel=1e-3):
        """y: packed counts (totM); i0, fro2: one float per slice."""
        n = self.n
        i0a = (ctypes.c_double * n)(*[float(v) for v in i0])
        fra = (ctypes.c_double * n)(*[float(v) for v in fro2])
        _check(_lib.dg_batch_bind(self._h, _ptr(y, torch.float32, self.totM, "y"), i0a, fra,
                                  _ptr(self.x, torch.float32), _ptr(self.s, torch.float32),
                                  _ptr(self.scal, torch.float64),
                                  _ptr(mu_out, torch.float32, self.totN, "mu_out"), int(den_kind),
                                  ctypes.cast(ctypes.pointer(den_params), ctypes.c_void_p),
                                  float(eps_rel), _ptr(self.work, torch.uint8)))
        self.keep = (y, den_params, mu_out)

    def state_init(self, tau_x0=1.0):
        _check(_lib.dg_batch_state_init(self._h, float(tau_x0), _stream()))

    def iterate(self, n_iter, t0=0, probe_seed=0, eta_x=1.0, eta_s=1.0, onsager=True,
                channel_mode=CHANNEL_LAPLACE, write_mu=False):
        _check(_lib.dgamp_batch_iterate(self._h, int(n_iter), int(t0), int(probe_seed),
                                        float(eta_x), float(eta_s), 1 if onsager else 0,
                                        int(channel_mode), 1 if write_mu else 0, _stream()))

    def autotune(self, reps=10):
        _check(_lib.dg_batch_autotune(self._h, int(reps), _stream()))
        return int(_lib.dg_batch_projector_variant(self._h))

    @property
    def projector_variant(self):
        return int(_lib.dg_batch_projector_variant(self._h))

    @projector_variant.setter
    def projector_variant(self, v):
        _check(_lib.dg_batch_set_projector_variant(self._h, int(v)))

    @property
    def nlm_variant(self):
        return int(_lib.dg_batch_nlm_variant(self._h))

    @nlm_variant.setter
    def nlm_variant(self, v):
        _check(_lib.dg_batch_set_nlm_variant(self._h, int(v)))

    def graph(self, n_iter, tau_x0=1.0, probe_seed=0, eta_x=1.0, eta_s=1.0, onsager=True,
              channel_mode=CHANNEL_LAPLACE):
        return BatchGraph(self, n_iter, tau_x0, probe_seed, eta_x, eta_s, onsager, channel_mode)

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _lib is not None:
                _lib.dg_batch_destroy(self._h)
                self._h = None
        except Exception:
            pass


class BatchGraph(DgampGraph):
    """A captured batched reconstruction (state reset + n_iter iterations + mu_out)."""

    def __init__(self, batch, n_iter, tau_x0, probe_seed, eta_x, eta_s, onsager, channel_mode):
        self.keep = batch
        h = _VP()
        _check(_lib.dg_batch_graph_create(batch._h, float(tau_x0), int(n_iter), int(probe_seed),
                                          float(eta_x), float(eta_s), 1 if onsager else 0,
                                          int(channel_mode), ctypes.byref(h)))
        self._h = h


class CnnNet:
    """Residual CNN denoiser state on the device: FP32 master parameters (PyTorch
    layout per layer: w[co][ci][3][3], b[co]), Adam moments and the packed BF16
    network the kernels read."""

    def __init__(self, master=None, seed=0):
        load()
        self.P = int(_lib.dg_cnn_param_count())
        if master is None:
            master = self.init_master(seed)
        master = torch.as_tensor(master, dtype=torch.float32).reshape(-1)
        if master.numel() != self.P:
            raise DgError("CNN parameter vector must have %d values" % self.P)
        self.master = master.cuda().contiguous()
        self.grad = torch.zeros_like(self.master)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.packed = torch.zeros(int(_lib.dg_cnn_weight_bytes()), dtype=torch.uint8, device="cuda")
        self.step = 0
        self._work = {}
        self.repack()

    @staticmethod
    def layer_shapes():
        s = [((64, 1, 3, 3), (64,))] + [((64, 64, 3, 3), (64,))] * 8 + [((1, 64, 3, 3), (1,))]
        return s

    @classmethod
    def init_master(cls, seed, scale=1.0):
        import numpy as np
        rng = np.random.default_rng(seed)
        parts = []
        for ws, bs in cls.layer_shapes():
            fan_in = ws[1] * 9
            parts.append((rng.standard_normal(ws) * np.sqrt(2.0 / fan_in) * scale).ravel())
            parts.append(np.zeros(bs))
        return np.concatenate(parts).astype(np.float32)

    def layers(self):
        """Host copy of the parameters as [(w, b), ...] (float64)."""
        flat = self.master.detach().cpu().double().numpy()
        out, k = [], 0
        for ws, bs in self.layer_shapes():
            nw, nb = int(np.prod(ws)), int(np.prod(bs))
            out.append((flat[k:k + nw].reshape(ws), flat[k + nw:k + nw + nb].reshape(bs)))
            k += nw + nb
        return out

    def repack(self):
        _check(_lib.dg_cnn_pack(_ptr(self.master, torch.float32, self.P, "master"),
                                _ptr(self.packed, torch.uint8, None, "packed"), _stream()))

    def work_for(self, n_pixels):
        if n_pixels not in self._work:
            nbytes = int(_lib.dg_cnn_workspace_bytes(int(n_pixels)))
            self._work[n_pixels] = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        return self._work[n_pixels]

    def forward(self, imgs):
        """D(imgs) for a (n, h, w) float32 CUDA tensor."""
        n, h, w = imgs.shape
        out = torch.empty_like(imgs)
        _check(_lib.dg_cnn_forward(_ptr(self.packed, torch.uint8, None, "packed"), n, h, w,
                                   _ptr(imgs, torch.float32, None, "in"),
                                   _ptr(out, torch.float32, None, "out"),
                                   _ptr(self.work_for(n * h * w), torch.uint8, None, "work"),
                                   _stream()))
        return out

    def train_step(self, noisy, clean, lr, loss_out=None):
        n, h, w = noisy.shape
        if loss_out is None:
            loss_out = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.step += 1
        _check(_lib.dg_cnn_train_step(_ptr(noisy, torch.float32, None, "noisy"),
                                      _ptr(clean, torch.float32, noisy.numel(), "clean"), n, h, w,
                                      _ptr(self.master, torch.float32, self.P, "master"),
                                      _ptr(self.packed, torch.uint8, None, "packed"),
                                      _ptr(self.grad, torch.float32, self.P, "grad"),
                                      _ptr(self.m, torch.float32, self.P, "m"),
                                      _ptr(self.v, torch.float32, self.P, "v"), self.step, float(lr),
                                      _ptr(loss_out, torch.float64, 1, "loss"),
                                      _ptr(self.work_for(n * h * w), torch.uint8, None, "work"),
                                      _stream()))
        return loss_out

    def save(self, path):
        from safetensors.torch import save_file
        save_file({"master": self.master.detach().cpu()}, path)

    @classmethod
    def load_file(cls, path):
        from safetensors.torch import load_file
        return cls(master=load_file(path)["master"])
