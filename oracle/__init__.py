"""FP64 CPU oracle of the Asp-Clean2016 minor cycle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package.  It is independent of the HIP library: the minor cycle
lives in plain C (``asp_oracle.c``, FP64, no fused multiply-add), the MLP of
the learned proposal in NumPy FP64 (``mlp.py``), and the smoothing initial
values with their switch in NumPy/SciPy FP64 (``smoothing.py``).  This module
marshals arguments to the C code and drives the switch.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_DIR, "asp_oracle.c")
_SO = os.path.join(_DIR, "libasp_oracle.so")

ORC_OK, ORC_STOP_THRESHOLD, ORC_STOP_MAXITER, ORC_LM_NOT_CONVERGED = 0, 1, 2, 3
MAX_ACTIVE = 16

COMP_DTYPE = np.dtype([("a", "<f8"), ("x", "<f8"), ("y", "<f8"), ("s", "<f8"),
                       ("iter_added", "<i8"), ("iter_updated", "<i8")])


# A build of the same source made elsewhere (the sanitizer test's
# AddressSanitizer/UBSan build) can stand in for the library.
_OVERRIDE = os.environ.get("ASP_ORACLE_LIB")
if _OVERRIDE:
    _SO = _OVERRIDE


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, -O2, no fast-math, no contraction)."""
    if _OVERRIDE:
        return _SO
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"], cwd=_DIR)
        os.replace(tmp, _SO)
    return _SO


class _Comp(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("x", ctypes.c_double), ("y", ctypes.c_double),
                ("s", ctypes.c_double), ("iter_added", ctypes.c_int64),
                ("iter_updated", ctypes.c_int64)]


class _State(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int64), ("W", ctypes.c_int64),
                ("gain", ctypes.c_double), ("threshold", ctypes.c_double),
                ("max_iter", ctypes.c_int64), ("max_active", ctypes.c_int32),
                ("lm_max_iter", ctypes.c_int32), ("max_width", ctypes.c_double),
                ("window_sigmas", ctypes.c_double),
                ("lm_mu0", ctypes.c_double), ("lm_tol", ctypes.c_double), ("alpha_b", ctypes.c_double),
                ("omega_b", ctypes.c_double), ("R", ctypes.POINTER(ctypes.c_double)),
                ("comps", ctypes.c_void_p), ("L", ctypes.c_int64), ("cap", ctypes.c_int64),
                ("k", ctypes.c_int64)]


class _Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_active", ctypes.c_int32),
                ("idx", ctypes.c_int64), ("peak", ctypes.c_double),
                ("members", ctypes.c_int32 * MAX_ACTIVE),
                ("lm_iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("used_fallback", ctypes.c_int32), ("start_from_proposal", ctypes.c_int32),
                ("chi2_init", ctypes.c_double), ("chi2_final", ctypes.c_double),
                ("theta", ctypes.c_double * (4 * MAX_ACTIVE)),
                ("theta0", ctypes.c_double * (4 * MAX_ACTIVE)),
                ("omega_px", ctypes.c_int64), ("update_px", ctypes.c_int64),
                ("added", ctypes.c_int32), ("pad", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        L.orc_default_config.argtypes = [ctypes.POINTER(_State)]
        L.orc_halfwidth.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_halfwidth.restype = ctypes.c_int
        L.orc_box.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                              ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.orc_peak.argtypes = [dp, ctypes.c_int64]
        L.orc_peak.restype = ctypes.c_int64
        L.orc_psf_fit.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int64)]
        L.orc_deconvolve.argtypes = [ctypes.c_double] * 4 + [ctypes.POINTER(ctypes.c_double)] * 3 + [
            ctypes.POINTER(ctypes.c_int32)]
        L.orc_convolve.argtypes = [ctypes.c_double] * 4 + [ctypes.POINTER(ctypes.c_double)] * 2
        L.orc_cholesky_solve.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_step.argtypes = [ctypes.POINTER(_State), ctypes.c_void_p, ctypes.POINTER(_Report),
                               ctypes.c_void_p]
        L.orc_step_start.argtypes = [ctypes.POINTER(_State), dp, ctypes.POINTER(_Report),
                                     ctypes.c_void_p]
        L.orc_run.argtypes = [ctypes.POINTER(_State), ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.orc_residual_from_scratch.argtypes = [ctypes.POINTER(_State), dp, dp]
        L.orc_fit_eval.argtypes = [ctypes.POINTER(_State), ctypes.c_int, dp, dp, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64)]
        L.orc_fit_eval.restype = ctypes.c_double
        L.orc_fit_gaussians.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, dp,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_double)]
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# Thin functional wrappers
# ---------------------------------------------------------------------------

def halfwidth(s: float, window_sigmas: float = 5.0) -> int:
    return lib().orc_halfwidth(s, window_sigmas)


def box(x: float, y: float, h: int, H: int, W: int):
    b = (ctypes.c_int64 * 4)()
    lib().orc_box(x, y, h, H, W, b)
    return tuple(b)


def peak(R: np.ndarray) -> int:
    R = np.ascontiguousarray(R, dtype=np.float64)
    return int(lib().orc_peak(R.ravel(), R.size))


def psf_fit(psf: np.ndarray, main_lobe_frac: float = 0.35):
    psf = np.ascontiguousarray(psf, dtype=np.float64)
    a, w, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    rc = lib().orc_psf_fit(psf.ravel(), psf.shape[0], psf.shape[1], main_lobe_frac,
                           ctypes.byref(a), ctypes.byref(w), ctypes.byref(n))
    if rc != 0:
        raise ValueError(f"orc_psf_fit failed: {rc}")
    return a.value, w.value, n.value


def deconvolve(a: float, s: float, alpha_b: float, omega_b: float):
    """Eqs. (5)-(6): (flux, alpha_i, omega_i, is_point) of a fitted Gaussian."""
    f, al, om, ip = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    lib().orc_deconvolve(a, s, alpha_b, omega_b, ctypes.byref(f), ctypes.byref(al),
                         ctypes.byref(om), ctypes.byref(ip))
    return f.value, al.value, om.value, bool(ip.value)


def convolve(alpha: float, omega: float, alpha_b: float, omega_b: float):
    a, s = ctypes.c_double(), ctypes.c_double()
    lib().orc_convolve(alpha, omega, alpha_b, omega_b, ctypes.byref(a), ctypes.byref(s))
    return a.value, s.value


def cholesky_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray | None:
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    rc = lib().orc_cholesky_solve(A.shape[0], A.ravel(), b, x)
    return None if rc != 0 else x


def fit_gaussians(data: np.ndarray, theta0, omega_b: float, max_width: float = 0.0,
                  window_sigmas: float = 5.0, lm_max_iter: int = 100, mu0: float = 1e-3,
                  tol: float = 1e-5):
    data = np.ascontiguousarray(data, dtype=np.float64)
    th = np.ascontiguousarray(np.asarray(theta0, dtype=np.float64).ravel().copy())
    conv, chi2 = ctypes.c_int32(), ctypes.c_double()
    trials = lib().orc_fit_gaussians(data.ravel(), data.shape[0], data.shape[1], th.size // 4, th,
                                     omega_b, max_width, window_sigmas, lm_max_iter, mu0, tol,
                                     ctypes.byref(conv), ctypes.byref(chi2))
    return th.reshape(-1, 4), trials, bool(conv.value), chi2.value


# ---------------------------------------------------------------------------
# Stateful minor cycle
# ---------------------------------------------------------------------------

class Oracle:
    """The FP64 minor cycle on a residual it owns.

    ``alpha_b``/``omega_b`` come from the PSF fit unless given (the lockstep
    harness passes the values under test so both sides start identical)."""

    def __init__(self, dirty, psf=None, *, gain=0.1, threshold=0.0, max_iter=1000,
                 max_active=5, cap=None, alpha_b=None, omega_b=None, lm_max_iter=100,
                 window_sigmas=5.0, lm_tol=1e-5, max_width=0.0, smooth_scales=0,
                 smooth_norm="peak", switch_deconvolved=False):
        L = lib()
        self.dirty = np.ascontiguousarray(dirty, dtype=np.float64)
        H, W = self.dirty.shape
        self.R = self.dirty.copy()
        if alpha_b is None or omega_b is None:
            alpha_b, omega_b, _ = psf_fit(psf)
        cap = int(cap if cap is not None else max_iter + 1)
        self.comps_buf = np.zeros(cap, dtype=COMP_DTYPE)
        st = _State()
        L.orc_default_config(ctypes.byref(st))
        st.H, st.W = H, W
        st.gain, st.threshold, st.max_iter = gain, threshold, max_iter
        st.max_active, st.lm_max_iter = max_active, lm_max_iter
        st.window_sigmas, st.lm_tol, st.max_width = window_sigmas, lm_tol, max_width
        st.alpha_b, st.omega_b = alpha_b, omega_b
        st.R = self.R.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        st.comps = self.comps_buf.ctypes.data
        st.L, st.cap, st.k = 0, cap, 0
        self.st = st
        # the smoothing method and its switch (Sect. 2 step 1, Sect. 3);
        # smooth_scales = 0 keeps the simple method in every iteration
        self.smooth_scales = int(smooth_scales)
        self.smooth_norm = smooth_norm
        self.switch_deconvolved = bool(switch_deconvolved)
        self.smooth_now = self.smooth_scales > 0

    @property
    def s_max(self) -> float:
        st = self.st
        m = st.max_width if st.max_width > 0.0 else min(st.H, st.W) / 8.0
        return max(m, st.omega_b)

    def smooth_best(self, method=None) -> dict:
        """The smoothing method's peak and start values on the current residual."""
        from . import smoothing
        return smoothing.best(self.R, self.st.omega_b, max(1, self.smooth_scales), self.s_max,
                              self.st.window_sigmas, method, self.smooth_norm)

    # -- state ------------------------------------------------------------
    @property
    def k(self) -> int:
        return int(self.st.k)

    @property
    def L(self) -> int:
        return int(self.st.L)

    @property
    def alpha_b(self) -> float:
        return self.st.alpha_b

    @property
    def omega_b(self) -> float:
        return self.st.omega_b

    def comps(self) -> np.ndarray:
        """(L, 4) array of convolved-space (a, x, y, s)."""
        c = self.comps_buf[: self.L]
        return np.stack([c["a"], c["x"], c["y"], c["s"]], axis=1)

    def load_state(self, R, comps, k, iter_added=None, iter_updated=None):
        """Overwrite the state: residual (any float dtype, converted exactly to
        FP64), component list (L, 4) and the iteration counter."""
        self.R[...] = np.asarray(R, dtype=np.float64).reshape(self.R.shape)
        comps = np.asarray(comps, dtype=np.float64).reshape(-1, 4)
        n = comps.shape[0]
        if n > self.comps_buf.shape[0]:
            raise ValueError("capacity")
        for i, f in enumerate("axys"):
            self.comps_buf[f][:n] = comps[:, i]
        self.comps_buf["iter_added"][:n] = 0 if iter_added is None else iter_added
        self.comps_buf["iter_updated"][:n] = 0 if iter_updated is None else iter_updated
        self.st.L = n
        self.st.k = int(k)

    # -- the iteration ----------------------------------------------------
    def step(self, init=None, want_hess=False, start=None, smooth=None) -> dict:
        """One iteration.  init: a proposal (learned mode).  With the smoothing
        method on, ``smooth`` (default: the switch's state) says whether this
        iteration smooths; ``start`` overrides the smoothing start values (a
        caller that checked a near-tie passes the other side's choice)."""
        from . import smoothing
        rep = _Report()
        hess = np.zeros((4 * MAX_ACTIVE) ** 2) if want_hess else None
        hp = None if hess is None else hess.ctypes.data
        use_smooth = self.smooth_now if smooth is None else bool(smooth)
        sb = None
        if self.smooth_scales > 0 and use_smooth and init is None:
            if start is None:
                sb = self.smooth_best()
                start = sb["start"]
            st4 = np.ascontiguousarray(np.asarray(start, dtype=np.float64))
            rc = lib().orc_step_start(ctypes.byref(self.st), st4, ctypes.byref(rep), hp)
        else:
            use_smooth = False
            ip = None
            if init is not None:
                init_arr = np.ascontiguousarray(np.asarray(init, dtype=np.float64))
                ip = init_arr.ctypes.data
            rc = lib().orc_step(ctypes.byref(self.st), ip, ctypes.byref(rep), hp)
        m = rep.n_active
        out = {"status": rc, "idx": int(rep.idx), "peak": rep.peak, "n_active": m,
               "members": list(rep.members[:m]), "lm_iters": rep.lm_iters,
               "converged": bool(rep.converged), "used_fallback": bool(rep.used_fallback),
               "start_from_proposal": bool(rep.start_from_proposal),
               "chi2_init": rep.chi2_init, "chi2_final": rep.chi2_final,
               "theta": np.array(rep.theta[: 4 * m]).reshape(-1, 4),
               "theta0": np.array(rep.theta0[: 4 * m]).reshape(-1, 4),
               "omega_px": int(rep.omega_px), "update_px": int(rep.update_px),
               "added": bool(rep.added)}
        if want_hess and m:
            n = 4 * m
            out["hess"] = hess[: n * n].reshape(n, n).copy()
        out["smoothed"] = use_smooth
        if sb is not None:
            out["smooth"] = {k: sb[k] for k in ("scale", "idx", "sigma", "score", "corr", "norm2")}
        if self.smooth_scales > 0 and rc in (ORC_OK, ORC_LM_NOT_CONVERGED):
            # the switch for the next iteration, from the new component's start
            # width and fitted width
            self.smooth_now = not smoothing.simple_next(
                float(out["theta"][0, 3]), float(out["theta0"][0, 3]), self.st.omega_b,
                self.switch_deconvolved)
        return out

    def run(self, n_iter: int):
        if self.smooth_scales > 0:
            rc, i = ORC_OK, 0
            for i in range(n_iter):
                rc = self.step()["status"]
                if rc not in (ORC_OK, ORC_LM_NOT_CONVERGED):
                    return rc, i
            return rc, n_iter
        done = ctypes.c_int64()
        rc = lib().orc_run(ctypes.byref(self.st), n_iter, ctypes.byref(done))
        return rc, done.value

    def fit_eval(self, theta, stored=None) -> dict:
        """One evaluation of the fit objective on the current residual: theta
        (m, 4) with the new component first, stored (m, 4) the old members'
        stored parameters (row 0 unused).  Returns F, H = J^T J, g = J^T (D - M),
        chi2 and the pixel count of U."""
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, 4))
        m = th.shape[0]
        sd = np.zeros_like(th) if stored is None else np.ascontiguousarray(
            np.asarray(stored, dtype=np.float64).reshape(m, 4))
        n = 4 * m
        H = np.zeros((n, n))
        g = np.zeros(n)
        chi2, npx = ctypes.c_double(), ctypes.c_int64()
        F = lib().orc_fit_eval(ctypes.byref(self.st), m, th.ravel(), sd.ravel(), H.ctypes.data,
                               g.ctypes.data, ctypes.byref(chi2), ctypes.byref(npx))
        return {"F": F, "H": H, "g": g, "chi2": chi2.value, "npx": int(npx.value)}

    def residual_from_scratch(self) -> np.ndarray:
        out = np.zeros_like(self.dirty)
        lib().orc_residual_from_scratch(ctypes.byref(self.st), self.dirty.ravel(), out.ravel())
        return out

    def components(self) -> list[dict]:
        """Deconvolved components (Eqs. 5-6) with the loop-gained amplitude."""
        res = []
        for a, x, y, s in self.comps():
            f, al, om, ip = deconvolve(a, s, self.alpha_b, self.omega_b)
            res.append({"flux": f, "amp": al, "x": x, "y": y, "width": om, "amp_c": a,
                        "width_c": s, "is_point": ip})
        return res
