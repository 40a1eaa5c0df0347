"""ctypes binding of libfrpmg.so (argument marshalling only).

Every computation happens in the HIP library; this module converts torch
tensors to device pointers, Python parameters to the C structs declared in
``include/frpmg.h`` and status codes to exceptions.  There is no fallback:
if the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfrpmg.so")

FR_OK, FR_EINVAL, FR_ENOMEM, FR_EDEVICE = 0, -1, -2, -3
FR_ESINGULAR, FR_ENOCONV, FR_EBREAKDOWN, FR_ENONFINITE = -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESINGULAR", -5: "ENOCONV",
                -6: "EBREAKDOWN", -7: "ENONFINITE"}
EPS_ABSOLUTE, EPS_NORMALIZED, EPS_SCALED = 0, 1, 2
FD_CENTRAL = 4  # ORed into an EPS_* mode: central difference
PREC_FP64, PREC_FP32, PREC_FP32_BF16, PREC_BF16_STORE = 0, 1, 2, 3
COARSE_NONE, COARSE_EJ, COARSE_LEARNED, COARSE_MBNK = 0, 1, 2, 3
SMOOTHER_EJ, SMOOTHER_MBNK = 0, 1
SCALE_LITERAL, SCALE_NORMALIZED, SCALE_SCALED = 0, 1, 2
SCHEME_ESDIRK, SCHEME_ROW = 0, 1
PRECOND_EJ, PRECOND_PMG, PRECOND_PMG_LEARNED = 0, 1, 2
MAX_LEVELS = 4
MAX_NEWTON_LOG = 128

EXPORTS = ["fr_create", "fr_destroy", "fr_last_error", "fr_level_size", "fr_residual", "fr_residual_noalloc",
           "fr_jvp", "ej_factor",
           "ej_solve", "ej_get_inverse", "pmg_restrict", "pmg_prolong", "pmg_set_point", "pmg_precond_apply",
           "gmres_solve_stage", "fr_time_step", "fr_step_tableau", "lcc_harvest", "lcc_harvest_count", "lcc_train", "lcc_dims", "lcc_num_weights",
           "lcc_get_weights", "lcc_set_weights", "lcc_get_scales", "lcc_set_scales", "lcc_forward",
           "lcc_loss_grad", "lcc_features_of", "lcc_adam_step", "mbnk_factor", "mbnk_matvec", "mbnk_ilu_solve", "mbnk_solve",
           "mbnk_get_blocks", "fr_pa_hierarchy", "fr_set_degrees", "fr_get_degrees", "fr_pa_indicator",
           "fr_pa_adapt", "fr_pa_project"]


class FRError(RuntimeError):
    def __init__(self, func, code, msg):
        super().__init__("%s failed: %s (%d): %s" % (func, STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.POINTER(ctypes.c_double) * 3),
                ("nlevels", ctypes.c_int), ("p", ctypes.c_int * MAX_LEVELS),
                ("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("Pr", ctypes.c_double),
                ("tau", ctypes.c_double), ("qinf", ctypes.c_double * 5)]


class PmgParams(ctypes.Structure):
    _fields_ = [("sigma_D", ctypes.c_double), ("n0", ctypes.c_int), ("n1", ctypes.c_int),
                ("coarse_mode", ctypes.c_int), ("scale_mode", ctypes.c_int), ("eps_p", ctypes.c_double),
                ("n2", ctypes.c_int), ("n3", ctypes.c_int), ("levels", ctypes.c_int),
                ("mbnk_maxit", ctypes.c_int), ("mbnk_tol", ctypes.c_double)]


class StageParams(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("a_ii", ctypes.c_double), ("a_i1", ctypes.c_double),
                ("dt", ctypes.c_double), ("dtau", ctypes.c_double), ("m", ctypes.c_int),
                ("max_restarts", ctypes.c_int), ("eta", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_ptc", ctypes.c_int), ("precond", ctypes.c_int), ("precision", ctypes.c_int),
                ("n0", ctypes.c_int), ("n1", ctypes.c_int), ("eps", ctypes.c_double),
                ("eps_mode", ctypes.c_int), ("scale_mode", ctypes.c_int), ("eps_p", ctypes.c_double),
                ("skip_setup", ctypes.c_int), ("stall_window", ctypes.c_int), ("stall_ratio", ctypes.c_double),
                ("graphs", ctypes.c_int), ("n2", ctypes.c_int), ("n3", ctypes.c_int),
                ("pmg_levels", ctypes.c_int), ("solver", ctypes.c_int), ("coarse_smoother", ctypes.c_int),
                ("mbnk_maxit", ctypes.c_int), ("mbnk_tol", ctypes.c_double), ("smoother_refresh", ctypes.c_int),
                ("verify", ctypes.c_int)]

SOLVER_JFNK, SOLVER_PMG = 0, 1


class LccHarvestParams(ctypes.Structure):
    _fields_ = [("enable", ctypes.c_int), ("max_pairs", ctypes.c_int), ("stride", ctypes.c_int),
                ("target_sweeps", ctypes.c_int), ("reset", ctypes.c_int)]


class LccTrainParams(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("holdout", ctypes.c_double), ("reinit", ctypes.c_int)]


class LccTrainStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("val_loss", ctypes.c_double), ("val_loss_init", ctypes.c_double), ("t_train", ctypes.c_double)]


class StageStats(ctypes.Structure):
    _fields_ = [("ptc_iters", ctypes.c_int), ("gmres_iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("converged", ctypes.c_int), ("status", ctypes.c_int),
                ("res0", ctypes.c_double), ("res", ctypes.c_double), ("rel_res", ctypes.c_double),
                ("true_rel_res", ctypes.c_double),
                ("t_total", ctypes.c_double), ("t_setup", ctypes.c_double), ("t_solve", ctypes.c_double),
                ("n_R_fine", ctypes.c_long), ("n_R_coarse", ctypes.c_long),
                ("n_ej_fine", ctypes.c_long), ("n_ej_coarse", ctypes.c_long),
                ("fallbacks", ctypes.c_int), ("gmres_per_newton", ctypes.c_int * MAX_NEWTON_LOG),
                ("t_precond", ctypes.c_double), ("t_jvp", ctypes.c_double), ("t_ortho", ctypes.c_double)]

    def as_dict(self):
        d = {f[0]: getattr(self, f[0]) for f in self._fields_ if f[0] != "gmres_per_newton"}
        n = self.ptc_iters if self.ptc_iters > 0 else 1
        d["gmres_per_newton"] = list(self.gmres_per_newton)[:min(n, MAX_NEWTON_LOG)]
        return d


TAB_ESDIRK3, TAB_ROW3, TAB_ESDIRK2, TAB_ROW2, TAB_ESDIRK4, TAB_ROW4 = 0, 1, 2, 3, 4, 5
MAX_STEP_STAGES = 5


class StepParams(ctypes.Structure):
    _fields_ = [("tableau", ctypes.c_int), ("stage", StageParams)]


class Tableau(ctypes.Structure):
    _fields_ = [("rosenbrock", ctypes.c_int), ("stages", ctypes.c_int), ("gamma", ctypes.c_double),
                ("A", (ctypes.c_double * 6) * 6), ("a", (ctypes.c_double * 4) * 4),
                ("c", (ctypes.c_double * 4) * 4), ("m", ctypes.c_double * 4)]


class StepStats(ctypes.Structure):
    _fields_ = [("nstages", ctypes.c_int), ("gmres_iters", ctypes.c_int), ("ptc_iters", ctypes.c_int),
                ("fallbacks", ctypes.c_int), ("status", ctypes.c_int),
                ("t_total", ctypes.c_double), ("t_setup", ctypes.c_double), ("t_solve", ctypes.c_double),
                ("n_R_fine", ctypes.c_long), ("n_R_coarse", ctypes.c_long),
                ("n_ej_fine", ctypes.c_long), ("n_ej_coarse", ctypes.c_long),
                ("stage", StageStats * MAX_STEP_STAGES)]

    def as_dict(self):
        d = {f[0]: getattr(self, f[0]) for f in self._fields_ if f[0] != "stage"}
        d["stages"] = [self.stage[i].as_dict() for i in range(self.nstages)]
        return d


_lib = None


def load():
    """Load libfrpmg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfrpmg.so is not built (run __graft_entry__.build() or "
                           "python -m paper_2202_09733_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.c_double
    L.fr_create.argtypes = [ctypes.POINTER(MeshDesc), ctypes.POINTER(ctypes.c_void_p)]
    L.fr_destroy.argtypes = [vp]
    L.fr_destroy.restype = None
    L.fr_last_error.argtypes = [vp]
    L.fr_last_error.restype = ctypes.c_char_p
    L.fr_level_size.argtypes = [vp, ctypes.c_int]
    L.fr_level_size.restype = ctypes.c_size_t
    L.fr_residual.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.fr_residual_noalloc.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.fr_pa_hierarchy.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
    L.fr_set_degrees.argtypes = [vp, vp, ctypes.c_int]
    L.fr_get_degrees.argtypes = [vp, ctypes.c_int, vp]
    L.fr_pa_indicator.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp, vp]
    L.fr_pa_adapt.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, dp, dp, vp]
    L.fr_pa_project.argtypes = [vp, vp, ctypes.c_int, vp, vp, ctypes.c_int, vp, vp]
    L.fr_jvp.argtypes = [vp, ctypes.c_int, vp, vp, vp, dp, dp, ctypes.c_int, vp, vp]
    L.ej_factor.argtypes = [vp, ctypes.c_int, vp, dp, ctypes.c_int, vp]
    L.ej_solve.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.ej_get_inverse.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    L.pmg_restrict.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    L.pmg_prolong.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    L.pmg_set_point.argtypes = [vp, vp, vp, vp]
    L.pmg_precond_apply.argtypes = [vp, ctypes.POINTER(PmgParams), vp, vp, vp]
    L.gmres_solve_stage.argtypes = [vp, ctypes.POINTER(StageParams), vp, vp, ctypes.POINTER(StageStats), vp]
    L.fr_time_step.argtypes = [vp, ctypes.POINTER(StepParams), vp, vp, ctypes.POINTER(StepStats), vp]
    L.fr_step_tableau.argtypes = [ctypes.c_int, ctypes.POINTER(Tableau)]
    ip = ctypes.POINTER(ctypes.c_int)
    fp = ctypes.POINTER(ctypes.c_float)
    L.lcc_harvest.argtypes = [vp, ctypes.POINTER(LccHarvestParams)]
    L.lcc_harvest_count.argtypes = [vp]
    L.lcc_train.argtypes = [vp, ctypes.POINTER(LccTrainParams), ctypes.POINTER(LccTrainStats), vp]
    L.lcc_dims.argtypes = [vp, ip, ip, ip, ip, ip]
    L.lcc_num_weights.argtypes = [vp]
    L.lcc_num_weights.restype = ctypes.c_size_t
    L.lcc_get_weights.argtypes = [vp, fp, ctypes.c_size_t]
    L.lcc_set_weights.argtypes = [vp, fp, ctypes.c_size_t]
    L.lcc_get_scales.argtypes = [vp, fp, fp]
    L.lcc_set_scales.argtypes = [vp, fp, fp]
    L.lcc_forward.argtypes = [vp, vp, ctypes.c_int, vp, vp]
    L.lcc_loss_grad.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), vp, vp]
    L.lcc_features_of.argtypes = [vp, vp, vp, vp, vp]
    L.lcc_adam_step.argtypes = [vp, vp, dp, vp]
    L.mbnk_factor.argtypes = [vp, ctypes.c_int, vp, dp, vp]
    L.mbnk_matvec.argtypes = [vp, vp, vp, vp]
    L.mbnk_ilu_solve.argtypes = [vp, vp, vp, vp]
    L.mbnk_solve.argtypes = [vp, vp, vp, dp, ctypes.c_int, vp]
    L.mbnk_get_blocks.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("fr_destroy", "fr_last_error", "fr_level_size", "lcc_num_weights"):
            f.restype = ctypes.c_int
    _lib = L
    return L


def step_tableau(tableau):
    """The coefficients the library's full time step uses for a tableau
    (host call, no device): a dict with gamma and either A (ESDIRK, s x s)
    or the transformed a, c, m (ROW)."""
    t = Tableau()
    rc = load().fr_step_tableau(int(tableau), ctypes.byref(t))
    if rc != FR_OK:
        raise FRError("fr_step_tableau", rc, "unknown tableau %r" % (tableau,))
    s = t.stages
    out = {"rosenbrock": bool(t.rosenbrock), "stages": s, "gamma": t.gamma}
    if t.rosenbrock:
        out["a"] = [[t.a[i][j] for j in range(s)] for i in range(s)]
        out["c"] = [[t.c[i][j] for j in range(s)] for i in range(s)]
        out["m"] = [t.m[i] for i in range(s)]
    else:
        out["A"] = [[t.A[i][j] for j in range(s)] for i in range(s)]
    return out


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    import torch
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), \
        "expected a contiguous float64 CUDA tensor"
    return ctypes.c_void_p(t.data_ptr())


def _iptr(t):
    import torch
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32 and t.is_contiguous(), \
        "expected a contiguous int32 CUDA tensor"
    return ctypes.c_void_p(t.data_ptr())


def nested_degrees(deg, nlevels, gap):
    """Per-element degrees of every p-sublevel, [nlevels][Ne] (fr_pa_hierarchy)."""
    d = np.ascontiguousarray(np.asarray(deg, dtype=np.int32))
    out = np.empty((nlevels, d.shape[0]), dtype=np.int32)
    rc = load().fr_pa_hierarchy(d.ctypes.data, d.shape[0], int(nlevels), int(gap), out.ctypes.data)
    if rc != FR_OK:
        raise FRError("fr_pa_hierarchy", rc, "bad degrees, level count or gap")
    return out


def _fptr(t):
    import torch
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous(), \
        "expected a contiguous float32 CUDA tensor"
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class StageConfig:
    scheme: int = SCHEME_ESDIRK
    a_ii: float = 0.43586652150845899942
    a_i1: float = 0.43586652150845899942
    dt: float = 1e-3
    dtau: float = 0.0
    m: int = 30
    max_restarts: int = 20
    eta: float = 0.1
    tol: float = 1e-8
    max_ptc: int = 100
    precond: int = PRECOND_PMG
    precision: int = PREC_FP64
    n0: int = 2
    n1: int = 2
    eps: float = 1e-6
    eps_mode: int = EPS_SCALED
    scale_mode: int = SCALE_SCALED
    eps_p: float = 1e-6
    skip_setup: int = 0
    stall_window: int = 0
    stall_ratio: float = 0.0
    graphs: int = 0
    n2: int = 2
    n3: int = 2
    pmg_levels: int = 0
    solver: int = 0
    coarse_smoother: int = SMOOTHER_EJ
    mbnk_maxit: int = 0
    mbnk_tol: float = 0.0
    smoother_refresh: int = 0
    verify: int = 1

    def to_c(self):
        return StageParams(**{f[0]: getattr(self, f[0]) for f in StageParams._fields_})


class FR:
    """One library context: a periodic mesh with a hierarchy of degrees."""

    def __init__(self, dim, n, h, levels, gamma, mu, Pr, tau, qinf, device="cuda:0"):
        import torch
        self.lib = load()
        self.device = torch.device(device)
        self.dim = int(dim)
        self.n = tuple(int(x) for x in n)
        self.levels = [int(p) for p in levels]
        self.nv = self.dim + 2
        self.Ne = int(np.prod(self.n))
        d = MeshDesc()
        d.dim = self.dim
        self._h = [np.ascontiguousarray(np.asarray(h[a], dtype=np.float64)) for a in range(self.dim)]
        for a in range(3):
            d.n[a] = self.n[a] if a < self.dim else 1
        for a in range(self.dim):
            d.h[a] = self._h[a].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.nlevels = len(self.levels)
        for i, p in enumerate(self.levels):
            d.p[i] = p
        d.gamma, d.mu, d.Pr, d.tau = gamma, mu, Pr, tau
        for v in range(self.nv):
            d.qinf[v] = float(qinf[v])
        h_ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.fr_create(ctypes.byref(d), ctypes.byref(h_ctx))
        if rc != FR_OK:
            raise FRError("fr_create", rc, "see stderr")
        self.ctx = h_ctx

    @classmethod
    def from_workload(cls, wl, levels=None, device="cuda:0"):
        levels = [wl.p0, wl.p1] if levels is None else levels
        return cls(wl.dim, wl.n, wl.h, levels, wl.gamma, wl.mu, wl.Pr, wl.tau, wl.qinf, device=device)

    @classmethod
    def from_padapt(cls, wl, deg, nlevels=2, gap=2, device="cuda:0"):
        """A context whose finest level has the degree map deg and whose
        coarser levels the nested degrees (fr_set_degrees)."""
        levels = [int(x) for x in nested_degrees(deg, nlevels, gap).max(axis=1)]
        fr = cls(wl.dim, wl.n, wl.h, levels, wl.gamma, wl.mu, wl.Pr, wl.tau, wl.qinf, device=device)
        fr.set_degrees(deg, gap)
        return fr

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.fr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ------------------------------------------------------------
    def _check(self, name, rc):
        if rc != FR_OK:
            raise FRError(name, rc, self.lib.fr_last_error(self.ctx).decode())

    def shape(self, level=0):
        P = self.levels[level] + 1
        return (self.nv, P ** self.dim, self.Ne)

    def empty(self, level=0):
        import torch
        return torch.empty(self.shape(level), dtype=torch.float64, device=self.device)

    def to_dev(self, a):
        import torch
        return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=self.device).contiguous()

    # -- ABI calls ------------------------------------------------------------
    def residual(self, level, dq, out=None):
        out = self.empty(level) if out is None else out
        self._check("fr_residual", self.lib.fr_residual(self.ctx, level, _ptr(dq), _ptr(out), _stream()))
        return out

    def residual_noalloc(self, level, dq, out=None):
        out = self.empty(level) if out is None else out
        self._check("fr_residual_noalloc", self.lib.fr_residual_noalloc(self.ctx, level, _ptr(dq), _ptr(out),
                                                                        _stream()))
        return out

    def jvp(self, level, dq, rq, v, shift, eps=1e-6, eps_mode=EPS_SCALED, out=None):
        out = self.empty(level) if out is None else out
        self._check("fr_jvp", self.lib.fr_jvp(self.ctx, level, _ptr(dq), _ptr(rq), _ptr(v), float(shift),
                                              float(eps), int(eps_mode), _ptr(out), _stream()))
        return out

    def ej_factor(self, level, dq_lin, sigma, precision=PREC_FP64):
        self._check("ej_factor", self.lib.ej_factor(self.ctx, level, _ptr(dq_lin), float(sigma),
                                                    int(precision), _stream()))

    def ej_solve(self, level, r, out=None):
        out = self.empty(level) if out is None else out
        self._check("ej_solve", self.lib.ej_solve(self.ctx, level, _ptr(r), _ptr(out), _stream()))
        return out

    def ej_inverse(self, level):
        """Stored inverse blocks as [Ne][nb][nb] row-major numpy (FP64)."""
        nb = self.nv * (self.levels[level] + 1) ** self.dim
        buf = np.empty(self.Ne * nb * nb)
        self._check("ej_get_inverse", self.lib.ej_get_inverse(
            self.ctx, level, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return buf.reshape(self.Ne, nb, nb).transpose(0, 2, 1).copy()

    def restrict(self, frm, x, out=None):
        out = self.empty(frm + 1) if out is None else out
        self._check("pmg_restrict", self.lib.pmg_restrict(self.ctx, frm, frm + 1, _ptr(x), _ptr(out), _stream()))
        return out

    def prolong(self, frm, x, out=None):
        out = self.empty(frm - 1) if out is None else out
        self._check("pmg_prolong", self.lib.pmg_prolong(self.ctx, frm, frm - 1, _ptr(x), _ptr(out), _stream()))
        return out

    def set_degrees(self, deg, gap=2):
        if deg is None:
            self._check("fr_set_degrees", self.lib.fr_set_degrees(self.ctx, None, int(gap)))
            return
        d = np.ascontiguousarray(np.asarray(deg, dtype=np.int32))
        assert d.shape == (self.Ne,)
        self._check("fr_set_degrees", self.lib.fr_set_degrees(self.ctx, d.ctypes.data, int(gap)))

    def get_degrees(self, level):
        out = np.empty(self.Ne, dtype=np.int32)
        self._check("fr_get_degrees", self.lib.fr_get_degrees(self.ctx, level, out.ctypes.data))
        return out

    def pa_indicator(self, level, dq, var=1, out=None):
        import torch
        out = torch.empty(self.Ne, dtype=torch.float64, device=self.device) if out is None else out
        self._check("fr_pa_indicator", self.lib.fr_pa_indicator(self.ctx, level, _ptr(dq), int(var), _ptr(out),
                                                                _stream()))
        return out

    def pa_adapt(self, eta, deg_in, p_max, p_min=1, nu_max=0.2, nu_min=0.001, out=None):
        import torch
        out = torch.empty(self.Ne, dtype=torch.int32, device=self.device) if out is None else out
        self._check("fr_pa_adapt", self.lib.fr_pa_adapt(self.ctx, _ptr(eta), _iptr(deg_in), _iptr(out), int(p_min),
                                                        int(p_max), float(nu_max), float(nu_min), _stream()))
        return out

    def pa_project(self, deg_from, p_from, x, deg_to, p_to, out=None):
        import torch
        if out is None:
            out = torch.empty((self.nv, (p_to + 1) ** self.dim, self.Ne), dtype=torch.float64, device=self.device)
        self._check("fr_pa_project", self.lib.fr_pa_project(self.ctx, _iptr(deg_from), int(p_from), _ptr(x),
                                                            _iptr(deg_to), int(p_to), _ptr(out), _stream()))
        return out

    def pmg_set_point(self, dq, rq):
        self._keep_point = (dq, rq)
        self._check("pmg_set_point", self.lib.pmg_set_point(self.ctx, _ptr(dq), _ptr(rq), _stream()))

    def pmg_apply(self, x, sigma_D, n0=2, n1=2, coarse_mode=COARSE_EJ, scale_mode=SCALE_SCALED, eps_p=1e-6,
                  out=None, n2=2, n3=2, levels=0, mbnk_maxit=0, mbnk_tol=0.0):
        out = self.empty(0) if out is None else out
        prm = PmgParams(float(sigma_D), int(n0), int(n1), int(coarse_mode), int(scale_mode), float(eps_p),
                        int(n2), int(n3), int(levels), int(mbnk_maxit), float(mbnk_tol))
        self._check("pmg_precond_apply", self.lib.pmg_precond_apply(self.ctx, ctypes.byref(prm), _ptr(x),
                                                                    _ptr(out), _stream()))
        return out

    # -- MBNK smoother ------------------------------------------------------------
    def mbnk_factor(self, level, dq_lin, sigma):
        self._mb_level = level
        self._check("mbnk_factor", self.lib.mbnk_factor(self.ctx, level, _ptr(dq_lin), float(sigma), _stream()))

    def mbnk_matvec(self, x, out=None):
        out = self.empty(self._mb_level) if out is None else out
        self._check("mbnk_matvec", self.lib.mbnk_matvec(self.ctx, _ptr(x), _ptr(out), _stream()))
        return out

    def mbnk_ilu_solve(self, r, out=None):
        out = self.empty(self._mb_level) if out is None else out
        self._check("mbnk_ilu_solve", self.lib.mbnk_ilu_solve(self.ctx, _ptr(r), _ptr(out), _stream()))
        return out

    def mbnk_solve(self, g, tol=0.1, maxit=5, out=None):
        out = self.empty(self._mb_level) if out is None else out
        self._check("mbnk_solve", self.lib.mbnk_solve(self.ctx, _ptr(g), _ptr(out), float(tol), int(maxit),
                                                      _stream()))
        return out

    def mbnk_blocks(self):
        """Assembled blocks as numpy: D [Ne][nb][nb], O [Ne][2 dim][nb][nb], row-major."""
        nb = self.nv * (self.levels[self._mb_level] + 1) ** self.dim
        D = np.empty(self.Ne * nb * nb)
        O = np.empty(self.Ne * 2 * self.dim * nb * nb)
        dp_ = ctypes.POINTER(ctypes.c_double)
        self._check("mbnk_get_blocks", self.lib.mbnk_get_blocks(self.ctx, D.ctypes.data_as(dp_),
                                                                O.ctypes.data_as(dp_)))
        D = D.reshape(self.Ne, nb, nb).transpose(0, 2, 1).copy()
        O = O.reshape(self.Ne, 2 * self.dim, nb, nb).transpose(0, 1, 3, 2).copy()
        return D, O

    # -- learned coarse correction ---------------------------------------------
    def lcc_dims(self):
        v = [ctypes.c_int() for _ in range(5)]
        self._check("lcc_dims", self.lib.lcc_dims(self.ctx, *[ctypes.byref(x) for x in v]))
        return dict(zip(["nin", "nin_pad", "nh", "nout", "nout_pad"], [x.value for x in v]))

    def lcc_harvest(self, enable=1, max_pairs=100000, stride=8, target_sweeps=8, reset=0):
        prm = LccHarvestParams(int(enable), int(max_pairs), int(stride), int(target_sweeps), int(reset))
        self._check("lcc_harvest", self.lib.lcc_harvest(self.ctx, ctypes.byref(prm)))

    def lcc_count(self):
        return int(self.lib.lcc_harvest_count(self.ctx))

    def lcc_train(self, epochs=20, batch=256, lr=1e-3, seed=7, holdout=0.1, reinit=0):
        prm = LccTrainParams(int(epochs), int(batch), float(lr), int(seed), float(holdout), int(reinit))
        st = LccTrainStats()
        self._check("lcc_train", self.lib.lcc_train(self.ctx, ctypes.byref(prm), ctypes.byref(st), _stream()))
        return {f[0]: getattr(st, f[0]) for f in LccTrainStats._fields_}

    def _wshapes(self):
        d = self.lcc_dims()
        return [(d["nh"], d["nin_pad"]), (d["nh"], d["nh"]), (d["nout_pad"], d["nh"])]

    def lcc_get_weights(self):
        n = int(self.lib.lcc_num_weights(self.ctx))
        buf = np.empty(n, dtype=np.float32)
        self._check("lcc_get_weights", self.lib.lcc_get_weights(
            self.ctx, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n))
        out, off = [], 0
        for r, c in self._wshapes():
            out.append(buf[off:off + r * c].reshape(r, c).copy())
            off += r * c
        return out

    def lcc_set_weights(self, Ws):
        buf = np.ascontiguousarray(np.concatenate([np.asarray(w, dtype=np.float32).reshape(-1) for w in Ws]))
        self._check("lcc_set_weights", self.lib.lcc_set_weights(
            self.ctx, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), buf.size))

    def lcc_get_scales(self):
        a = np.zeros(self.nv, dtype=np.float32)
        b = np.zeros(self.nv, dtype=np.float32)
        self._check("lcc_get_scales", self.lib.lcc_get_scales(
            self.ctx, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            b.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return a, b

    def lcc_set_scales(self, in_scale, out_scale):
        a = np.ascontiguousarray(in_scale, dtype=np.float32)
        b = np.ascontiguousarray(out_scale, dtype=np.float32)
        self._check("lcc_set_scales", self.lib.lcc_set_scales(
            self.ctx, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            b.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def lcc_forward(self, X):
        import torch
        d = self.lcc_dims()
        Xd = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32), device=self.device).contiguous()
        Y = torch.empty((X.shape[0], d["nout_pad"]), dtype=torch.float32, device=self.device)
        self._check("lcc_forward", self.lib.lcc_forward(self.ctx, _fptr(Xd), int(X.shape[0]), _fptr(Y), _stream()))
        return Y.cpu().numpy()

    def lcc_loss_grad(self, X, T):
        import torch
        Xd = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32), device=self.device).contiguous()
        Td = torch.as_tensor(np.ascontiguousarray(T, dtype=np.float32), device=self.device).contiguous()
        n = int(self.lib.lcc_num_weights(self.ctx))
        g = torch.empty(n, dtype=torch.float32, device=self.device)
        loss = ctypes.c_double()
        self._check("lcc_loss_grad", self.lib.lcc_loss_grad(self.ctx, _fptr(Xd), _fptr(Td), int(X.shape[0]),
                                                            ctypes.byref(loss), _fptr(g), _stream()))
        gh = g.cpu().numpy()
        out, off = [], 0
        for r, c in self._wshapes():
            out.append(gh[off:off + r * c].reshape(r, c).copy())
            off += r * c
        return loss.value, out

    def lcc_adam_step(self, grads, lr):
        """One Adam step of the master weights with the given per-layer gradients."""
        import torch
        g = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.float32).reshape(-1) for x in grads]))
        gd = torch.as_tensor(g, device=self.device).contiguous()
        self._check("lcc_adam_step", self.lib.lcc_adam_step(self.ctx, _fptr(gd), float(lr), _stream()))
        torch.cuda.synchronize(self.device)

    def lcc_features_of(self, d1):
        import torch
        d = self.lcc_dims()
        rows = torch.empty((self.Ne, d["nin_pad"]), dtype=torch.float32, device=self.device)
        s = torch.empty(self.Ne, dtype=torch.float32, device=self.device)
        self._check("lcc_features_of", self.lib.lcc_features_of(self.ctx, _ptr(d1), _fptr(rows), _fptr(s),
                                                                _stream()))
        return rows.cpu().numpy(), s.cpu().numpy()

    def solve_stage(self, cfg: StageConfig, dq_n, out=None, raise_on_noconv=True):
        out = self.empty(0) if out is None else out
        st = StageStats()
        prm = cfg.to_c()
        rc = self.lib.gmres_solve_stage(self.ctx, ctypes.byref(prm), _ptr(dq_n), _ptr(out), ctypes.byref(st),
                                        _stream())
        if rc != FR_OK and (raise_on_noconv or rc != FR_ENOCONV):
            self._check("gmres_solve_stage", rc)
        d = st.as_dict()
        d["rc"] = rc
        return out, d

    def time_step(self, cfg: StageConfig, dq_n, tableau=TAB_ESDIRK3, out=None, raise_on_noconv=True):
        """One full time step (every stage); cfg gives dt and the solver settings."""
        out = self.empty(0) if out is None else out
        st = StepStats()
        prm = StepParams(tableau=tableau, stage=cfg.to_c())
        rc = self.lib.fr_time_step(self.ctx, ctypes.byref(prm), _ptr(dq_n), _ptr(out), ctypes.byref(st),
                                   _stream())
        if rc != FR_OK and (raise_on_noconv or rc != FR_ENOCONV):
            self._check("fr_time_step", rc)
        d = st.as_dict()
        d["rc"] = rc
        return out, d


def stage_config_for(wl, precond=PRECOND_PMG, precision=PREC_FP64, **kw):
    """Stage parameters of a workload (ESDIRK: second stage, a_21 = a_22)."""
    scheme = SCHEME_ESDIRK if wl.scheme == "esdirk" else SCHEME_ROW
    eta = 0.1 if precond != PRECOND_EJ else 0.01
    cfg = StageConfig(scheme=scheme, a_ii=wl.a_ii, a_i1=wl.a_ii, dt=wl.dt, dtau=wl.dt, precond=precond,
                      precision=precision, eta=eta)
    for k, v in kw.items():
        setattr(cfg, k, v)
    return cfg
