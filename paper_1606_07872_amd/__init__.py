"""Python binding of the gfx950 Asp-Clean2016 minor cycle (``include/asp.h``).

Argument marshalling only: every step of the minor cycle runs in the HIP
kernels of ``libasp.so``.  Loading fails loudly when the library has not been
built (``python -m paper_1606_07872_amd.build``); there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libasp.so")

ASP_OK, ASP_STOP_THRESHOLD, ASP_STOP_MAXITER, ASP_LM_NOT_CONVERGED = 0, 1, 2, 3
ASP_ERR_INVALID_ARG, ASP_ERR_NONFINITE, ASP_ERR_PSF, ASP_ERR_STATE = -1, -2, -3, -4
ASP_ERR_CAPACITY, ASP_ERR_DEVICE, ASP_ERR_NOMEM = -5, -6, -7
MAX_ACTIVE = 16
MAX_SCALES = 8

# Every symbol include/asp.h declares.
EXPORTS = ["asp_default_options", "asp_create", "asp_create_device", "asp_destroy",
           "asp_last_error", "asp_find_peak", "asp_fit_active_set", "asp_update_residual",
           "asp_last_fit", "asp_eval_trial", "asp_find_peak_noalloc", "asp_fit_histogram",
           "asp_step", "asp_run", "asp_components", "asp_components_raw", "asp_residual",
           "asp_residual_device", "asp_psf_gauss", "asp_counts", "asp_fit_profile",
           "asp_kernel_timing", "asp_kernel_times", "asp_set_mlp", "asp_set_init_mode",
           "asp_record", "asp_record_count", "asp_mlp_create", "asp_mlp_destroy",
           "asp_mlp_last_error", "asp_mlp_loss_grad", "asp_mlp_train", "asp_mlp_forward",
           "asp_mlp_weights", "asp_residual_sumsq", "asp_residual_sumsq_tracked", "asp_batch_create", "asp_batch_destroy",
           "asp_batch_last_error", "asp_batch_field", "asp_batch_config", "asp_batch_get_config",
           "asp_batch_run", "asp_batch_autotune", "asp_smooth_peak", "asp_smooth_map",
           "asp_smooth_widths", "asp_smooth_work", "asp_refresh_residual", "asp_step_2004",
           "asp_run_2004", "asp_model_image", "asp_state_size", "asp_save_state",
           "asp_load_state", "asp_set_2004_convolution"]

MLP_PARAMS = 329220
MLP_IN = 1024
MLP_OUT = 4


class AspError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"asp status {status}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("max_active", ctypes.c_int32), ("lm_max_iter", ctypes.c_int32),
                ("init_mode", ctypes.c_int32), ("capacity", ctypes.c_int32),
                ("fit_solo_tiles", ctypes.c_int32), ("fit_min_tiles", ctypes.c_int32),
                ("fit_group", ctypes.c_int32), ("smooth_scales", ctypes.c_int32),
                ("smooth_norm", ctypes.c_int32), ("switch_area", ctypes.c_int32),
                ("peak_tiles", ctypes.c_int32), ("refresh_every", ctypes.c_int32),
                ("update_launch", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("window_sigmas", ctypes.c_double), ("max_width", ctypes.c_double),
                ("lm_mu0", ctypes.c_double), ("lm_tol", ctypes.c_double),
                ("psf_lobe_frac", ctypes.c_double), ("stream", ctypes.c_void_p)]


class Gauss(ctypes.Structure):
    _fields_ = [("amp", ctypes.c_double), ("x", ctypes.c_double), ("y", ctypes.c_double),
                ("width", ctypes.c_double)]


class Component(ctypes.Structure):
    _fields_ = [("flux", ctypes.c_double), ("amp", ctypes.c_double), ("x", ctypes.c_double),
                ("y", ctypes.c_double), ("width", ctypes.c_double), ("amp_c", ctypes.c_double),
                ("width_c", ctypes.c_double), ("is_point", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("iter_added", ctypes.c_int64),
                ("iter_updated", ctypes.c_int64)]


class FitReport(ctypes.Structure):
    _fields_ = [("n_active", ctypes.c_int32), ("members", ctypes.c_int32 * MAX_ACTIVE),
                ("lm_iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("used_fallback", ctypes.c_int32), ("idx", ctypes.c_int64),
                ("peak", ctypes.c_float), ("pad", ctypes.c_float),
                ("chi2_init", ctypes.c_double), ("chi2_final", ctypes.c_double),
                ("theta0", ctypes.c_double * (4 * MAX_ACTIVE)),
                ("theta", ctypes.c_double * (4 * MAX_ACTIVE)),
                ("fit_px", ctypes.c_int64), ("init_source", ctypes.c_int32),
                ("start_from_proposal", ctypes.c_int32), ("init", ctypes.c_double * 4),
                ("added", ctypes.c_int32), ("pad2", ctypes.c_int32)]


class Fit2004Report(ctypes.Structure):
    _fields_ = [("idx", ctypes.c_int64), ("peak", ctypes.c_float), ("scale", ctypes.c_int32),
                ("trials", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("evaluations", ctypes.c_int32), ("direct_evals", ctypes.c_int32),
                ("start", ctypes.c_double * 4), ("theta0", ctypes.c_double * 4),
                ("theta", ctypes.c_double * 4), ("lo", ctypes.c_double * 4),
                ("hi", ctypes.c_double * 4), ("chi2_init", ctypes.c_double),
                ("chi2_final", ctypes.c_double), ("direct_update", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class BatchReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("fields_stopped", ctypes.c_int64),
                ("fields_failed", ctypes.c_int64), ("ms", ctypes.c_double)]


class RunReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("total_iterations", ctypes.c_int64),
                ("components", ctypes.c_int64), ("lm_trials", ctypes.c_int64),
                ("not_converged", ctypes.c_int64), ("fallbacks", ctypes.c_int64),
                ("pixels_updated", ctypes.c_int64), ("pixels_evaluated", ctypes.c_int64),
                ("gram_flops", ctypes.c_int64), ("smoothed", ctypes.c_int64),
                ("peak_tiles_scanned", ctypes.c_int64), ("not_added", ctypes.c_int64)]


COMPONENT_DTYPE = np.dtype([("flux", "<f8"), ("amp", "<f8"), ("x", "<f8"), ("y", "<f8"),
                            ("width", "<f8"), ("amp_c", "<f8"), ("width_c", "<f8"),
                            ("is_point", "<i4"), ("pad", "<i4"), ("iter_added", "<i8"),
                            ("iter_updated", "<i8")])

_lib = None


def lib():
    """The loaded C library; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run python -m paper_1606_07872_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, f32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_float, ctypes.c_double
        P = ctypes.POINTER
        L.asp_default_options.argtypes = [P(Options)]
        L.asp_create.argtypes = [vp, i64, i64, vp, i64, i64, f32, f32, P(Options), P(vp)]
        L.asp_create_device.argtypes = L.asp_create.argtypes
        L.asp_destroy.argtypes = [vp]
        L.asp_destroy.restype = None
        L.asp_last_error.argtypes = [vp]
        L.asp_last_error.restype = ctypes.c_char_p
        L.asp_find_peak.argtypes = [vp, P(i64), P(f32)]
        L.asp_fit_active_set.argtypes = [vp, i64, P(Gauss), P(FitReport)]
        L.asp_update_residual.argtypes = [vp, P(i64)]
        L.asp_last_fit.argtypes = [vp, P(FitReport)]
        L.asp_fit_histogram.argtypes = [vp, vp, vp, vp, ctypes.c_int32]
        L.asp_find_peak_noalloc.argtypes = [vp, i64, i64, vp, vp, vp]
        L.asp_eval_trial.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, P(f64), P(f64), P(i64)]
        L.asp_step.argtypes = [vp]
        L.asp_run.argtypes = [vp, i64, P(RunReport)]
        L.asp_components.argtypes = [vp, vp, i64, P(i64)]
        L.asp_components_raw.argtypes = [vp, vp, i64, P(i64)]
        L.asp_residual.argtypes = [vp, vp]
        L.asp_residual_device.argtypes = [vp, P(vp)]
        L.asp_psf_gauss.argtypes = [vp, P(f64), P(f64)]
        L.asp_counts.argtypes = [vp, P(i64), P(i64)]
        L.asp_kernel_timing.argtypes = [vp, ctypes.c_int32]
        L.asp_kernel_times.argtypes = [vp, vp, vp, ctypes.c_int32]
        L.asp_set_mlp.argtypes = [vp, vp, i64]
        L.asp_set_init_mode.argtypes = [vp, ctypes.c_int32]
        L.asp_record.argtypes = [vp, vp, vp, vp, i64]
        L.asp_record_count.argtypes = [vp, P(i64)]
        L.asp_mlp_create.argtypes = [vp, ctypes.c_int32, vp, P(vp)]
        L.asp_mlp_destroy.argtypes = [vp]
        L.asp_mlp_destroy.restype = None
        L.asp_mlp_last_error.argtypes = [vp]
        L.asp_mlp_last_error.restype = ctypes.c_char_p
        L.asp_mlp_loss_grad.argtypes = [vp, vp, vp, ctypes.c_int32, P(f64), vp]
        L.asp_mlp_train.argtypes = [vp, vp, vp, i64, vp, i64, ctypes.c_int32, f32, P(f64)]
        L.asp_mlp_forward.argtypes = [vp, vp, i64, vp]
        L.asp_mlp_weights.argtypes = [vp, vp]
        L.asp_residual_sumsq.argtypes = [vp, P(f64)]
        L.asp_residual_sumsq_tracked.argtypes = [vp, P(f64)]
        i32 = ctypes.c_int32
        L.asp_batch_create.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, P(Options), P(vp)]
        L.asp_batch_destroy.argtypes = [vp]
        L.asp_batch_destroy.restype = None
        L.asp_batch_last_error.argtypes = [vp]
        L.asp_batch_last_error.restype = ctypes.c_char_p
        L.asp_batch_field.argtypes = [vp, i32, P(vp)]
        L.asp_batch_config.argtypes = [vp, i32, i32, i32]
        L.asp_batch_get_config.argtypes = [vp, P(i32), P(i32), P(i32), P(i32)]
        L.asp_batch_run.argtypes = [vp, i64, P(BatchReport)]
        L.asp_batch_autotune.argtypes = [vp, i64, P(i32), P(i32), P(i32)]
        L.asp_fit_profile.argtypes = [vp, vp, ctypes.c_int32]
        L.asp_smooth_peak.argtypes = [vp, P(i32), P(i64), P(f32), P(Gauss)]
        L.asp_smooth_map.argtypes = [vp, i32, vp]
        L.asp_smooth_widths.argtypes = [vp, vp, i32, P(i32)]
        L.asp_smooth_work.argtypes = [vp, P(i64), P(f64)]
        L.asp_refresh_residual.argtypes = [vp]
        L.asp_step_2004.argtypes = [vp, P(Fit2004Report)]
        L.asp_model_image.argtypes = [vp, vp]
        L.asp_state_size.argtypes = [vp, P(i64)]
        L.asp_save_state.argtypes = [vp, vp, i64, P(i64)]
        L.asp_load_state.argtypes = [vp, vp, i64]
        L.asp_run_2004.argtypes = [vp, i64, P(RunReport)]
        L.asp_set_2004_convolution.argtypes = [vp, i32]
        for name in EXPORTS:
            if name not in ("asp_destroy", "asp_last_error", "asp_mlp_destroy",
                            "asp_mlp_last_error", "asp_batch_destroy", "asp_batch_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def default_options(**kw) -> Options:
    opt = Options()
    lib().asp_default_options(ctypes.byref(opt))
    for k, v in kw.items():
        if not hasattr(opt, k):
            raise TypeError(f"unknown option {k}")
        setattr(opt, k, v)
    return opt


def _is_device_tensor(a) -> bool:
    return hasattr(a, "is_cuda") and a.is_cuda


class Context:
    """One deconvolution context (``asp_ctx``).  ``dirty`` and ``psf`` are
    float32 host arrays (NumPy or CPU tensors), or float32 device tensors, in
    which case ``asp_create_device`` copies them device to device."""

    def __init__(self, dirty, psf, gain: float, threshold: float, **options):
        self._ctx = ctypes.c_void_p()
        opt = default_options(**options)
        if _is_device_tensor(dirty):
            if not _is_device_tensor(psf):
                raise TypeError("dirty and psf must both be device tensors or both host arrays")
            d, p = dirty.contiguous(), psf.contiguous()
            if str(d.dtype) != "torch.float32" or str(p.dtype) != "torch.float32":
                raise TypeError("float32 tensors required")
            H, W = d.shape
            Hp, Wp = p.shape
            rc = lib().asp_create_device(d.data_ptr(), H, W, p.data_ptr(), Hp, Wp, gain,
                                         threshold, ctypes.byref(opt), ctypes.byref(self._ctx))
        else:
            d = np.ascontiguousarray(np.asarray(dirty, dtype=np.float32))
            p = np.ascontiguousarray(np.asarray(psf, dtype=np.float32))
            H, W = d.shape
            Hp, Wp = p.shape
            rc = lib().asp_create(d.ctypes.data, H, W, p.ctypes.data, Hp, Wp, gain, threshold,
                                  ctypes.byref(opt), ctypes.byref(self._ctx))
        if rc != ASP_OK:
            raise AspError(rc, "asp_create failed")
        self.H, self.W = int(H), int(W)
        self.options = opt

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if self._ctx:
            lib().asp_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc):
        """Negative statuses raise; stops (> 0) are returned."""
        if rc < 0:
            raise AspError(rc, lib().asp_last_error(self._ctx).decode())
        return rc

    # -- the step API ------------------------------------------------------
    def find_peak(self):
        idx, val = ctypes.c_int64(), ctypes.c_float()
        rc = self._check(lib().asp_find_peak(self._ctx, ctypes.byref(idx), ctypes.byref(val)))
        return rc, idx.value, val.value

    def fit_active_set(self, idx: int, init=None):
        rep = FitReport()
        g = None
        if init is not None:
            g = Gauss(*[float(v) for v in init])
        rc = self._check(lib().asp_fit_active_set(self._ctx, idx, ctypes.byref(g) if g else None,
                                                   ctypes.byref(rep)))
        return rc, report_dict(rep)

    def last_fit(self) -> dict:
        """The report of the last fit (step API, run or batch)."""
        rep = FitReport()
        self._check(lib().asp_last_fit(self._ctx, ctypes.byref(rep)))
        return report_dict(rep)

    def eval_trial(self, theta, stored=None) -> dict:
        """One evaluation of the fit objective on the device (asp_eval_trial):
        theta (m, 4), stored (m, 4) with row 0 unused.  Returns F, H = J^T J,
        g = J^T (D - M), chi2 and the pixel count of U."""
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, 4))
        m = th.shape[0]
        sd = np.zeros_like(th) if stored is None else np.ascontiguousarray(
            np.asarray(stored, dtype=np.float64).reshape(m, 4))
        n = 4 * m
        H = np.zeros((n, n))
        g = np.zeros(n)
        F, chi2, npx = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        self._check(lib().asp_eval_trial(self._ctx, m, th.ctypes.data, sd.ctypes.data,
                                         H.ctypes.data, g.ctypes.data, ctypes.byref(F),
                                         ctypes.byref(chi2), ctypes.byref(npx)))
        return {"F": F.value, "H": H, "g": g, "chi2": chi2.value, "npx": int(npx.value)}

    def update_residual(self) -> int:
        n = ctypes.c_int64()
        self._check(lib().asp_update_residual(self._ctx, ctypes.byref(n)))
        return n.value

    def step(self) -> int:
        return self._check(lib().asp_step(self._ctx))

    def run(self, n_iter: int):
        rep = RunReport()
        rc = self._check(lib().asp_run(self._ctx, n_iter, ctypes.byref(rep)))
        return rc, {f: getattr(rep, f) for f, _ in RunReport._fields_}

    # -- state -------------------------------------------------------------
    def counts(self):
        k, L = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().asp_counts(self._ctx, ctypes.byref(k), ctypes.byref(L)))
        return k.value, L.value

    def components(self) -> np.ndarray:
        _, L = self.counts()
        out = np.zeros(max(L, 1), dtype=COMPONENT_DTYPE)
        n = ctypes.c_int64()
        self._check(lib().asp_components(self._ctx, out.ctypes.data, L, ctypes.byref(n)))
        return out[:L]

    def components_raw(self) -> np.ndarray:
        _, L = self.counts()
        out = np.zeros((max(L, 1), 4), dtype=np.float64)
        n = ctypes.c_int64()
        self._check(lib().asp_components_raw(self._ctx, out.ctypes.data, L, ctypes.byref(n)))
        return out[:L]

    def residual(self) -> np.ndarray:
        out = np.empty((self.H, self.W), dtype=np.float32)
        self._check(lib().asp_residual(self._ctx, out.ctypes.data))
        return out

    def residual_rms(self) -> float:
        """sqrt(mean residual^2), reduced on the device in FP64."""
        v = ctypes.c_double()
        self._check(lib().asp_residual_sumsq(self._ctx, ctypes.byref(v)))
        return float(np.sqrt(v.value / (self.H * self.W)))

    def residual_sumsq(self, tracked: bool = False) -> float:
        """Sum of residual^2 in FP64: a full pass (which also re-bases the
        tracked sum), or with tracked=True the sum kept up to date by the
        windowed updates, read without a pass over the image."""
        v = ctypes.c_double()
        f = lib().asp_residual_sumsq_tracked if tracked else lib().asp_residual_sumsq
        self._check(f(self._ctx, ctypes.byref(v)))
        return v.value

    def residual_device_ptr(self) -> int:
        p = ctypes.c_void_p()
        self._check(lib().asp_residual_device(self._ctx, ctypes.byref(p)))
        return p.value

    PROFILE_FIELDS = ("checkin_us", "setup_us", "eval_us", "wait_us", "reduce_us", "lmstep_us",
                      "commit_us", "prepare_us", "arrive_us", "trials", "fits", "eval_px",
                      "solo_trials", "solo_px")

    def fit_profile(self) -> dict:
        out = np.zeros(len(self.PROFILE_FIELDS))
        self._check(lib().asp_fit_profile(self._ctx, out.ctypes.data, len(out)))
        return dict(zip(self.PROFILE_FIELDS, out.tolist()))

    def fit_histogram(self) -> dict:
        """Per active-set size m: fits, LM trials and device microseconds."""
        n = MAX_ACTIVE + 1
        fits = np.zeros(n, dtype=np.int64)
        trials = np.zeros(n, dtype=np.int64)
        us = np.zeros(n)
        self._check(lib().asp_fit_histogram(self._ctx, fits.ctypes.data, trials.ctypes.data,
                                            us.ctypes.data, n))
        return {"fits": fits, "trials": trials, "us": us}

    KERNEL_KINDS = ("peak", "fit", "update", "propose", "smooth_passes", "smooth_pick",
                    "refresh", "eval2004", "update2004")

    def kernel_timing(self, on: bool):
        """Record HIP events around every launch of run()/step() (clears totals)."""
        self._check(lib().asp_kernel_timing(self._ctx, 1 if on else 0))

    def kernel_times(self) -> dict:
        """{kind: (total ms, launches)} from the recorded event pairs."""
        k = len(self.KERNEL_KINDS)
        ms = np.zeros(k)
        n = np.zeros(k, dtype=np.int64)
        self._check(lib().asp_kernel_times(self._ctx, ms.ctypes.data, n.ctypes.data, k))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(self.KERNEL_KINDS)}

    # -- learned start values ------------------------------------------------
    def set_mlp(self, weights):
        """Give the context the proposal network (flat FP32 weights, see Mlp)."""
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).ravel())
        self._check(lib().asp_set_mlp(self._ctx, w.ctypes.data, w.size))

    def set_init_mode(self, mode: int):
        """0 simple initial values, 1 the network's proposal, 2 the smoothing
        method with the 5 % switch."""
        self._check(lib().asp_set_init_mode(self._ctx, int(mode)))

    # -- the smoothing method ------------------------------------------------
    def smooth_peak(self) -> dict:
        """The smoothing method's peak on the current residual: scale j, pixel,
        |score| (FP32, as compared) and the start (a, x, y, s)."""
        j, idx, sc, g = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_float(), Gauss()
        self._check(lib().asp_smooth_peak(self._ctx, ctypes.byref(j), ctypes.byref(idx),
                                          ctypes.byref(sc), ctypes.byref(g)))
        return {"scale": j.value, "idx": idx.value, "score": sc.value,
                "start": np.array([g.amp, g.x, g.y, g.width])}

    def smooth_map(self, scale: int) -> np.ndarray:
        """The smoothed residual of trial width `scale` (H x W float32)."""
        out = np.empty((self.H, self.W), dtype=np.float32)
        self._check(lib().asp_smooth_map(self._ctx, int(scale), out.ctypes.data))
        return out

    def refresh_residual(self):
        """Replace the residual by I_dirty - B (*) I_model with the true PSF."""
        self._check(lib().asp_refresh_residual(self._ctx))

    def model_image(self) -> np.ndarray:
        """I_model: the components rendered in the sky plane (H x W float32)."""
        out = np.empty((self.H, self.W), dtype=np.float32)
        self._check(lib().asp_model_image(self._ctx, out.ctypes.data))
        return out

    # -- checkpoint and resume -------------------------------------------------
    def save_state(self) -> bytes:
        n = ctypes.c_int64()
        self._check(lib().asp_state_size(self._ctx, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(lib().asp_save_state(self._ctx, buf, n.value, ctypes.byref(n)))
        return buf.raw[: n.value]

    def load_state(self, blob: bytes):
        b = ctypes.create_string_buffer(bytes(blob), len(blob))
        self._check(lib().asp_load_state(self._ctx, b, len(blob)))

    # -- the Asp-Clean2004 comparison path -------------------------------------
    def step_2004(self):
        """One Asp-Clean2004 iteration (Eq. 3 fitted with the true PSF)."""
        rep = Fit2004Report()
        rc = self._check(lib().asp_step_2004(self._ctx, ctypes.byref(rep)))
        out = {}
        for f, _ in Fit2004Report._fields_:
            v = getattr(rep, f)
            out[f] = np.array(v[:]) if isinstance(v, ctypes.Array) else v
        return rc, out

    def set_2004_convolution(self, mode):
        """How the 2004 path forms B (*) g: "auto" (0), "fft" (1) or "direct" (2)."""
        code = {"auto": 0, "fft": 1, "direct": 2}.get(mode, mode)
        self._check(lib().asp_set_2004_convolution(self._ctx, int(code)))

    def run_2004(self, n_iter: int):
        rep = RunReport()
        rc = self._check(lib().asp_run_2004(self._ctx, n_iter, ctypes.byref(rep)))
        return rc, {f: getattr(rep, f) for f, _ in RunReport._fields_}

    def smooth_work(self):
        """(pixels, flops) of the smoothing passes since creation."""
        px, fl = ctypes.c_int64(), ctypes.c_double()
        self._check(lib().asp_smooth_work(self._ctx, ctypes.byref(px), ctypes.byref(fl)))
        return px.value, fl.value

    def smooth_widths(self) -> np.ndarray:
        out = np.zeros(MAX_SCALES)
        n = ctypes.c_int32()
        self._check(lib().asp_smooth_widths(self._ctx, out.ctypes.data, MAX_SCALES,
                                            ctypes.byref(n)))
        return out[: n.value]

    def record(self, patches, targets, flags):
        """Record a (patch, target, flag) triple per iteration into device tensors
        of shapes (cap, 1024) f32, (cap, 4) f32 and (cap,) int32; None turns it off."""
        if patches is None:
            self._check(lib().asp_record(self._ctx, None, None, None, 0))
            self._rec = None
            return
        cap = int(patches.shape[0])
        if tuple(patches.shape) != (cap, MLP_IN) or tuple(targets.shape) != (cap, MLP_OUT) \
                or tuple(flags.shape) != (cap,):
            raise ValueError("record buffers must be (cap, 1024), (cap, 4) and (cap,)")
        for t, dt in ((patches, "float32"), (targets, "float32"), (flags, "int32")):
            if not (_is_device_tensor(t) and str(t.dtype).endswith(dt) and t.is_contiguous()):
                raise ValueError("record buffers must be contiguous device tensors")
        self._rec = (patches, targets, flags)        # keep them alive
        self._check(lib().asp_record(self._ctx, patches.data_ptr(), targets.data_ptr(),
                                     flags.data_ptr(), cap))

    def record_count(self) -> int:
        n = ctypes.c_int64()
        self._check(lib().asp_record_count(self._ctx, ctypes.byref(n)))
        return n.value

    def psf_gauss(self):
        a, w = ctypes.c_double(), ctypes.c_double()
        self._check(lib().asp_psf_gauss(self._ctx, ctypes.byref(a), ctypes.byref(w)))
        return a.value, w.value


class Batch:
    """Many independent fields deconvolved by one persistent, graph-captured
    launch.  fields: a list of (dirty, psf, gain, threshold) with host float32
    images.  field(i) returns a Context view of field i."""

    def __init__(self, fields, **options):
        n = len(fields)
        opt = default_options(**options)
        self._keep = []
        dptr = (ctypes.c_void_p * n)()
        pptr = (ctypes.c_void_p * n)()
        H = (ctypes.c_int64 * n)()
        W = (ctypes.c_int64 * n)()
        Hp = (ctypes.c_int64 * n)()
        Wp = (ctypes.c_int64 * n)()
        gain = (ctypes.c_float * n)()
        thr = (ctypes.c_float * n)()
        for i, (dirty, psf, g, t) in enumerate(fields):
            d = np.ascontiguousarray(dirty, dtype=np.float32)
            q = np.ascontiguousarray(psf, dtype=np.float32)
            self._keep += [d, q]
            dptr[i], pptr[i] = d.ctypes.data, q.ctypes.data
            H[i], W[i] = d.shape
            Hp[i], Wp[i] = q.shape
            gain[i], thr[i] = float(g), float(t)
        self._b = ctypes.c_void_p()
        rc = lib().asp_batch_create(n, dptr, H, W, pptr, Hp, Wp, gain, thr, ctypes.byref(opt),
                                    ctypes.byref(self._b))
        if rc != ASP_OK:
            raise AspError(rc, "asp_batch_create failed")
        self._keep = None
        self.n = n
        self.shapes = [(int(H[i]), int(W[i])) for i in range(n)]

    def close(self):
        if self._b:
            lib().asp_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc < 0:
            raise AspError(rc, lib().asp_batch_last_error(self._b).decode())
        return rc

    def field(self, i: int) -> "Context":
        c = ctypes.c_void_p()
        self._check(lib().asp_batch_field(self._b, int(i), ctypes.byref(c)))
        ctx = Context.__new__(Context)
        ctx._ctx = c
        ctx.H, ctx.W = self.shapes[i]
        ctx._owner = self
        ctx.close = lambda: None            # the batch owns it
        return ctx

    def config(self, team_size=0, solo_tiles=0, min_tiles=0):
        self._check(lib().asp_batch_config(self._b, int(team_size), int(solo_tiles),
                                           int(min_tiles)))

    def get_config(self) -> dict:
        v = [ctypes.c_int32() for _ in range(4)]
        self._check(lib().asp_batch_get_config(self._b, *[ctypes.byref(x) for x in v]))
        return dict(zip(("team_size", "solo_tiles", "min_tiles", "grid"), [x.value for x in v]))

    def run(self, n_iter: int) -> dict:
        r = BatchReport()
        self._check(lib().asp_batch_run(self._b, int(n_iter), ctypes.byref(r)))
        return {f: getattr(r, f) for f, _ in BatchReport._fields_}

    def autotune(self, probe_iter: int = 10) -> dict:
        v = [ctypes.c_int32() for _ in range(3)]
        self._check(lib().asp_batch_autotune(self._b, int(probe_iter),
                                             *[ctypes.byref(x) for x in v]))
        return dict(zip(("team_size", "solo_tiles", "min_tiles"), [x.value for x in v]))


class Mlp:
    """The proposal network's trainer on the device (forward and backward passes
    and Adam by the library's kernels).  Inputs are contiguous FP32 device
    tensors; weights come in and go out as flat host arrays."""

    def __init__(self, weights, max_batch: int = 512, stream=None):
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).ravel())
        if w.size != MLP_PARAMS:
            raise ValueError(f"expected {MLP_PARAMS} weights")
        self._n = ctypes.c_void_p()
        rc = lib().asp_mlp_create(w.ctypes.data, int(max_batch),
                                  None if stream is None else ctypes.c_void_p(stream),
                                  ctypes.byref(self._n))
        if rc != ASP_OK:
            raise AspError(rc, "asp_mlp_create failed")
        self.max_batch = int(max_batch)

    def close(self):
        if self._n:
            lib().asp_mlp_destroy(self._n)
            self._n = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc < 0:
            raise AspError(rc, lib().asp_mlp_last_error(self._n).decode())
        return rc

    @staticmethod
    def _dev(t, cols, dtype="float32"):
        if not (_is_device_tensor(t) and str(t.dtype).endswith(dtype) and t.is_contiguous()):
            raise ValueError("expected a contiguous device tensor")
        if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
            raise ValueError(f"expected {cols} columns")
        return t.data_ptr()

    def loss_grad(self, x, t):
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        self._check(lib().asp_mlp_loss_grad(self._n, self._dev(x, MLP_IN), self._dev(t, MLP_OUT),
                                            int(x.shape[0]), ctypes.byref(loss), g.ctypes.data))
        return loss.value, g

    def train(self, x, t, order, batch: int, lr: float = 1e-3) -> float:
        """Adam steps over the rows of x, t picked by `order` (device int32 tensor,
        n_steps x batch indices); returns the mean batch loss."""
        n_steps = int(order.numel()) // int(batch)
        loss = ctypes.c_double()
        self._check(lib().asp_mlp_train(self._n, self._dev(x, MLP_IN), self._dev(t, MLP_OUT),
                                        int(x.shape[0]), self._dev(order, None, "int32"),
                                        n_steps, int(batch), float(lr), ctypes.byref(loss)))
        return loss.value

    def forward(self, x, y):
        self._check(lib().asp_mlp_forward(self._n, self._dev(x, MLP_IN), int(x.shape[0]),
                                          self._dev(y, MLP_OUT)))

    def weights(self) -> np.ndarray:
        w = np.zeros(MLP_PARAMS, dtype=np.float32)
        self._check(lib().asp_mlp_weights(self._n, w.ctypes.data))
        return w


def report_dict(rep: FitReport) -> dict:
    m = rep.n_active
    return {"n_active": m, "members": list(rep.members[:m]), "lm_iters": rep.lm_iters,
            "converged": bool(rep.converged), "used_fallback": bool(rep.used_fallback),
            "idx": rep.idx, "peak": rep.peak, "chi2_init": rep.chi2_init,
            "chi2_final": rep.chi2_final,
            "theta0": np.array(rep.theta0[: 4 * m]).reshape(-1, 4),
            "theta": np.array(rep.theta[: 4 * m]).reshape(-1, 4), "fit_px": rep.fit_px,
            "init_source": rep.init_source, "init": np.array(rep.init[:4]),
            "start_from_proposal": bool(rep.start_from_proposal), "added": bool(rep.added)}


# The C names, for callers that prefer them.
def asp_create(dirty, psf, gain, threshold, **options) -> Context:
    return Context(dirty, psf, gain, threshold, **options)
