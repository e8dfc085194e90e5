"""Thin Python binding of libfids (include/fids.h).

Argument marshalling only: every step of the time-stepping path runs in the
library's HIP kernels.  PyTorch provides device memory (the workspace and the
caller's arrays) and the HIP stream.  If libfids.so is missing the import of
this module succeeds but every call raises RuntimeError -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfids.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fids.h")

FIDS_OK, FIDS_EINVAL, FIDS_EDEVICE, FIDS_ENOCONV, FIDS_ENUMERIC, FIDS_ESTATE = 0, -1, -2, -3, -4, -5
FIDS_BICGSTAB, FIDS_FGMRES, FIDS_PCG = 0, 1, 2
FIDS_FP64, FIDS_MIXED = 0, 1
FIDS_STRANG, FIDS_NONE, FIDS_STRANG_K = 0, 1, 2
FIDS_HISTORY_SOE, FIDS_HISTORY_DIRECT = 0, 1
FIDS_LEVEL_ABOVE_TOL = 1


class Params(ctypes.Structure):
    _fields_ = [
        ("alpha", ctypes.c_double), ("gamma", ctypes.c_double), ("l", ctypes.c_double),
        ("T", ctypes.c_double), ("n", ctypes.c_int64), ("M", ctypes.c_int64),
        ("r", ctypes.c_double), ("mu", ctypes.c_double), ("soe_tol", ctypes.c_double),
        ("krylov_tol", ctypes.c_double), ("krylov_maxit", ctypes.c_int32),
        ("restart", ctypes.c_int32), ("solver", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("precond", ctypes.c_int32), ("kappa_time_dependent", ctypes.c_int32),
        ("x0_mode", ctypes.c_int32), ("store_states", ctypes.c_int32), ("wg_count", ctypes.c_int32),
        ("soe_helpers", ctypes.c_int32), ("history", ctypes.c_int32), ("checkpoint_every", ctypes.c_int32),
        ("dims", ctypes.c_int32),
    ]


def natural_len(params) -> int:
    """Unknowns per level: n, or n * n for dims = 2 (the caller's array length)."""
    return int(params.n) ** 2 if int(params.dims) == 2 else int(params.n)


def toeplitz_len(params) -> int:
    """Order of the Toeplitz matrix the library applies: n, or S (n - 1) + n
    for dims = 2 (rows of stride S, the smallest power of two >= 2n - 1)."""
    n = int(params.n)
    if int(params.dims) != 2:
        return n
    S = 1
    while S < 2 * n - 1:
        S *= 2
    return S * (n - 1) + n


class StepInfo(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("iters", ctypes.c_int32), ("matvecs", ctypes.c_int32),
                ("relres", ctypes.c_double), ("pc_fp64_iters", ctypes.c_int32), ("flags", ctypes.c_int32)]


class FidsError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        detail = ""
        if status == FIDS_EDEVICE:
            try:
                detail = " [" + lib().fids_last_error().decode() + "]"
            except Exception:
                pass
        super().__init__(f"{where}: {strerror(status)} ({status}){detail}")


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "fids_params_default": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "fids_workspace_size": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]),
    "fids_init_problem": (ctypes.c_int, [ctypes.POINTER(Params), _P, _P, _P, _P, ctypes.c_size_t, _P,
                                         ctypes.POINTER(_P)]),
    "fids_step": (ctypes.c_int, [_P, _P, ctypes.POINTER(StepInfo)]),
    "fids_solve_all": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(StepInfo)]),
    "fids_solve_levels": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.POINTER(StepInfo)]),
    "fids_solve_static": (ctypes.c_int, [ctypes.POINTER(Params), _P, _P, _P, _P, ctypes.POINTER(StepInfo), _P]),
    "fids_adjoint": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "fids_adjoint_report": (ctypes.c_int, [_P, ctypes.POINTER(StepInfo)]),
    "fids_precond_symbol": (ctypes.c_int, [_P, ctypes.c_int64, _D, _D]),
    "fids_reset": (ctypes.c_int, [_P]),
    "fids_prepare": (ctypes.c_int, [_P]),
    "fids_destroy": (ctypes.c_int, [_P]),
    "fids_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "fids_last_error": (ctypes.c_char_p, []),
    "fids_batch_workspace_size": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "fids_batch_init": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32, ctypes.POINTER(_P),
                                       ctypes.POINTER(_P), ctypes.POINTER(_P), _P, ctypes.c_size_t, _P,
                                       ctypes.POINTER(_P)]),
    "fids_batch_step": (ctypes.c_int, [_P, ctypes.POINTER(StepInfo)]),
    "fids_batch_solve_all": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(StepInfo)]),
    "fids_batch_solve_levels": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.POINTER(_P), ctypes.POINTER(StepInfo)]),
    "fids_batch_status": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]),
    "fids_batch_groups": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "fids_batch_tune": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "fids_batch_plan": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_double)]),
    "fids_batch_reset": (ctypes.c_int, [_P]),
    "fids_batch_prepare": (ctypes.c_int, [_P]),
    "fids_batch_destroy": (ctypes.c_int, [_P]),
    "fids_soe_nodes": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int32, _D, _D, ctypes.POINTER(ctypes.c_int32)]),
    "fids_ifl_column": (ctypes.c_int, [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]),
    "fids_ifl2d_mu": (ctypes.c_int, [ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "fids_ifl2d_coefficients": (ctypes.c_int, [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                               _D]),
    "fids_strang_eigs": (ctypes.c_int, [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]),
    "fids_level_coefficients": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                               ctypes.c_double, _D]),
    "fids_direct_weights": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_double,
                                           ctypes.c_int64, _D]),
}


def lib():
    """Load libfids.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2002_11978_amd.build`")
        # torch's wheel carries its own HIP runtime (same soname, different
        # file).  Loading torch first makes libfids bind to that runtime;
        # loading libfids first would put a second HIP and HSA runtime in the
        # process, and device pointers and streams would cross between them.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/fids.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(fids_\w+)\s*\(", txt, re.M)))


def strerror(status: int) -> str:
    try:
        return lib().fids_strerror(status).decode()
    except RuntimeError:
        return f"status {status}"


def _check(status, where):
    if status != FIDS_OK:
        raise FidsError(status, where)


def default_params(**kw) -> Params:
    p = Params()
    _check(lib().fids_params_default(ctypes.byref(p)), "fids_params_default")
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def workspace_size(p: Params) -> int:
    sz = ctypes.c_size_t(0)
    _check(lib().fids_workspace_size(ctypes.byref(p), ctypes.byref(sz)), "fids_workspace_size")
    return sz.value


# ------------------------------------------------------------------ host-only helpers
def _dptr(a):
    return a.ctypes.data_as(_D)


def soe_nodes(gamma, delta, T, tol, cap=4096):
    import numpy as np
    s = np.zeros(cap)
    w = np.zeros(cap)
    cnt = ctypes.c_int32(0)
    _check(lib().fids_soe_nodes(gamma, delta, T, tol, cap, _dptr(s), _dptr(w), ctypes.byref(cnt)),
           "fids_soe_nodes")
    return s[: cnt.value].copy(), w[: cnt.value].copy()


def ifl_column(n, alpha, l=1.0, mu=0.0):
    import numpy as np
    out = np.zeros(n)
    _check(lib().fids_ifl_column(n, alpha, l, mu, _dptr(out)), "fids_ifl_column")
    return out


def ifl2d_mu(alpha):
    out = ctypes.c_double(0.0)
    _check(lib().fids_ifl2d_mu(alpha, ctypes.byref(out)), "fids_ifl2d_mu")
    return out.value


def ifl2d_coefficients(n, alpha, l=1.0, mu=0.0):
    """a[p, q] (numpy, n x n) of the 2-D matrix, as the library builds it."""
    import numpy as np
    out = np.zeros(n * n)
    _check(lib().fids_ifl2d_coefficients(n, alpha, l, mu, _dptr(out)), "fids_ifl2d_coefficients")
    return out.reshape(n, n).T.copy()      # stored a[p + n q]: rows q -> transpose to [p, q]


def strang_eigs(n, alpha, l=1.0, mu=0.0):
    import numpy as np
    out = np.zeros(n)
    _check(lib().fids_strang_eigs(n, alpha, l, mu, _dptr(out)), "fids_strang_eigs")
    return out


def batch_plan(params, resident):
    """(group sizes, slots, modelled makespan) of a batch on `resident` workgroups (host only)."""
    count = len(params)
    arr = (Params * count)(*params)
    ng = (ctypes.c_int32 * count)()
    slot = (ctypes.c_int32 * count)()
    mk = ctypes.c_double(0.0)
    _check(lib().fids_batch_plan(arr, count, resident, ng, slot, ctypes.byref(mk)), "fids_batch_plan")
    return list(ng), list(slot), mk.value


def direct_weights(gamma, T, M, r, m):
    import numpy as np
    out = np.zeros(m)
    _check(lib().fids_direct_weights(gamma, T, M, r, m, _dptr(out)), "fids_direct_weights")
    return out


def level_coefficients(gamma, T, M, r):
    import numpy as np
    out = np.zeros(M)
    _check(lib().fids_level_coefficients(gamma, T, M, r, _dptr(out)), "fids_level_coefficients")
    return out


# ------------------------------------------------------------------ device problems
def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def solve_static(params: Params, kappa, f, phi, stream=None):
    """fids_solve_static: one allocation-free solve to level M (the library's
    fixed device array as workspace); returns (u^M, reports)."""
    import torch
    for name, t in (("kappa", kappa), ("f", f), ("phi", phi)):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float64 device tensor")
    s = stream if stream is not None else torch.cuda.current_stream(kappa.device)
    uT = torch.empty(natural_len(params), dtype=torch.float64, device=kappa.device)
    infos = (StepInfo * int(params.M))()
    _check(lib().fids_solve_static(ctypes.byref(params), _ptr(kappa), _ptr(f), _ptr(phi), _ptr(uT), infos,
                                   ctypes.c_void_p(s.cuda_stream)), "fids_solve_static")
    return uT, [LevelReport.of(i) for i in infos]


@dataclass
class LevelReport:
    m: int
    iters: int
    matvecs: int
    relres: float
    pc_fp64_iters: int = 0
    flags: int = 0

    @classmethod
    def of(cls, i):
        return cls(i.m, i.iters, i.matvecs, i.relres, i.pc_fp64_iters, i.flags)


class Problem:
    """One problem of eq. (1.1) on the current CUDA (HIP) device.

    kappa, f, phi are float64 device tensors in the layouts of fids.h; they
    are borrowed (kept referenced here) for the lifetime of the handle.
    """

    def __init__(self, params: Params, kappa, f, phi, stream=None):
        import torch
        self.torch = torch
        self.params = params
        for name, t in (("kappa", kappa), ("f", f), ("phi", phi)):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 device tensor")
        self.kappa, self.f, self.phi = kappa, f, phi
        self.device = kappa.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ws_bytes = workspace_size(params)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p(0)
        _check(lib().fids_init_problem(ctypes.byref(params), _ptr(kappa), _ptr(f), _ptr(phi), _ptr(self.ws),
                                       self.ws_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(h)), "fids_init_problem")
        self.h = h

    @property
    def n(self):
        """Unknowns per level (n, or n * n for dims = 2)."""
        return natural_len(self.params)

    @property
    def M(self):
        return int(self.params.M)

    def step(self):
        u = self.torch.empty(self.n, dtype=self.torch.float64, device=self.device)
        info = StepInfo()
        _check(lib().fids_step(self.h, _ptr(u), ctypes.byref(info)), "fids_step")
        return u, LevelReport.of(info)

    def solve_levels(self, count, want_u=True):
        """Advance `count` levels in one launch; returns (u at the new level, reports)."""
        u = self.torch.empty(self.n, dtype=self.torch.float64, device=self.device) if want_u else None
        infos = (StepInfo * count)()
        st = lib().fids_solve_levels(self.h, count, _ptr(u), infos)
        self.last_reports = [LevelReport.of(i) for i in infos if i.m > 0]
        _check(st, "fids_solve_levels")
        return u, self.last_reports

    def solve_levels_raw(self, count, u=None, infos=None):
        """fids_solve_levels with caller-provided outputs (no allocation); returns the status."""
        return lib().fids_solve_levels(self.h, count, _ptr(u), infos)

    def solve_all(self, return_all=False, want_uT=True):
        torch = self.torch
        uT = torch.empty(self.n, dtype=torch.float64, device=self.device) if want_uT else None
        uall = torch.empty((self.M + 1, self.n), dtype=torch.float64, device=self.device) if return_all else None
        infos = (StepInfo * self.M)()
        st = lib().fids_solve_all(self.h, _ptr(uT), _ptr(uall), infos)
        self.last_reports = [LevelReport.of(i) for i in infos]
        _check(st, "fids_solve_all")
        return uT, uall, self.last_reports

    def solve_all_raw(self, uT=None, uall=None, infos=None):
        """Like solve_all with caller-provided outputs (no allocation)."""
        return lib().fids_solve_all(self.h, _ptr(uT), _ptr(uall), infos)

    def adjoint(self, dJ_duT, g_kappa=None, g_f=None, g_phi=None, allocate=True):
        """dJ/dkappa, dJ/df, dJ/dphi for a loss J(u^M) with gradient dJ_duT.

        Outputs left as None are allocated when `allocate` is true, else
        not computed.
        """
        torch = self.torch
        if allocate:
            if g_kappa is None:
                g_kappa = torch.empty_like(self.kappa)
            if g_f is None:
                g_f = torch.empty((self.M, self.n), dtype=torch.float64, device=self.device)
            if g_phi is None:
                g_phi = torch.empty(self.n, dtype=torch.float64, device=self.device)
        for name, t in (("dJ_duT", dJ_duT), ("g_kappa", g_kappa), ("g_f", g_f), ("g_phi", g_phi)):
            if t is not None and not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 device tensor")
        _check(lib().fids_adjoint(self.h, _ptr(dJ_duT), _ptr(g_kappa), _ptr(g_f), _ptr(g_phi)), "fids_adjoint")
        return g_kappa, g_f, g_phi

    def adjoint_reports(self):
        infos = (StepInfo * self.M)()
        _check(lib().fids_adjoint_report(self.h, infos), "fids_adjoint_report")
        return [LevelReport.of(i) for i in infos]

    def reset(self):
        _check(lib().fids_reset(self.h), "fids_reset")

    def prepare(self):
        _check(lib().fids_prepare(self.h), "fids_prepare")

    def precond_symbol(self, m):
        """(q, qhat) of level m's Strang preconditioner as built on the device (host arrays)."""
        import numpy as np
        nt = toeplitz_len(self.params)
        L = 1
        while L < 2 * nt:
            L *= 2
        L = max(L, 4)
        q = np.zeros(nt)
        qhat = np.zeros(L // 2 + 1)
        _check(lib().fids_precond_symbol(self.h, m, _dptr(q), _dptr(qhat)), "fids_precond_symbol")
        return q, qhat

    def close(self):
        if getattr(self, "h", None):
            lib().fids_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent problems of eq. (1.1) advanced together (one workgroup
    each, one launch per solve or per level).

    params: list of Params (all with the same M); kappas, fs, phis: lists of
    float64 device tensors, borrowed for the lifetime of the batch.
    """

    def __init__(self, params, kappas, fs, phis, stream=None):
        import torch
        self.torch = torch
        count = len(params)
        if not (len(kappas) == len(fs) == len(phis) == count) or count < 1:
            raise ValueError("params, kappas, fs and phis must have the same nonzero length")
        for lst in (kappas, fs, phis):
            for t in lst:
                if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                    raise ValueError("batch arrays must be contiguous float64 device tensors")
        self.count = count
        self.params = (Params * count)(*params)
        self.kappas, self.fs, self.phis = list(kappas), list(fs), list(phis)
        self.device = kappas[0].device
        self.M = int(params[0].M)
        self.ns = [natural_len(p) for p in params]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nb = ctypes.c_size_t(0)
        _check(lib().fids_batch_workspace_size(self.params, count, ctypes.byref(nb)), "fids_batch_workspace_size")
        self.ws_bytes = nb.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        arr = lambda ts: (_P * count)(*[t.data_ptr() for t in ts])
        h = ctypes.c_void_p(0)
        _check(lib().fids_batch_init(self.params, count, arr(self.kappas), arr(self.fs), arr(self.phis),
                                     _ptr(self.ws), self.ws_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(h)), "fids_batch_init")
        self.h = h

    def _reports(self, infos):
        return [[LevelReport.of(i) for i in infos[p * self.M:(p + 1) * self.M]]
                for p in range(self.count)]

    def solve_all(self, want_uT=True):
        torch = self.torch
        outs = [torch.empty(n, dtype=torch.float64, device=self.device) for n in self.ns] if want_uT else None
        ptrs = (_P * self.count)(*[t.data_ptr() for t in outs]) if want_uT else None
        infos = (StepInfo * (self.count * self.M))()
        st = lib().fids_batch_solve_all(self.h, ptrs, infos)
        self.last_reports = self._reports(infos)
        _check(st, "fids_batch_solve_all")
        return outs, self.last_reports

    def solve_all_raw(self, uT_ptrs=None, infos=None):
        return lib().fids_batch_solve_all(self.h, uT_ptrs, infos)

    def solve_levels(self, count, want_u=True):
        """Advance every member `count` levels in one launch; returns (states, reports so far)."""
        torch = self.torch
        outs = [torch.empty(n, dtype=torch.float64, device=self.device) for n in self.ns] if want_u else None
        ptrs = (_P * self.count)(*[t.data_ptr() for t in outs]) if want_u else None
        infos = (StepInfo * (self.count * self.M))()
        st = lib().fids_batch_solve_levels(self.h, count, ptrs, infos)
        self.last_reports = self._reports(infos)
        _check(st, "fids_batch_solve_levels")
        return outs, self.last_reports

    def step(self):
        infos = (StepInfo * self.count)()
        _check(lib().fids_batch_step(self.h, infos), "fids_batch_step")
        return [LevelReport.of(i) for i in infos]

    def status(self):
        st = (ctypes.c_int32 * self.count)()
        last = (ctypes.c_int64 * self.count)()
        _check(lib().fids_batch_status(self.h, st, last), "fids_batch_status")
        return list(st), list(last)

    def tune(self, levels=4):
        """Autotune the tile shapes per class of members; returns each member's columns per tile."""
        ct = (ctypes.c_int32 * self.count)()
        _check(lib().fids_batch_tune(self.h, levels, ct), "fids_batch_tune")
        return list(ct)

    def groups(self):
        ng = (ctypes.c_int32 * self.count)()
        _check(lib().fids_batch_groups(self.h, ng), "fids_batch_groups")
        return list(ng)

    def reset(self):
        _check(lib().fids_batch_reset(self.h), "fids_batch_reset")

    def prepare(self):
        _check(lib().fids_batch_prepare(self.h), "fids_batch_prepare")

    def close(self):
        if getattr(self, "h", None):
            lib().fids_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
