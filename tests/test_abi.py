"""The C-ABI library loads and exports every symbol include/asp.h declares;
host-side argument checks.  CPU only: no call here reaches the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1606_07872_amd as asp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "asp.h")).read()
    return sorted(set(re.findall(r"\b(asp_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert header_symbols() == sorted(asp.EXPORTS)


def test_library_exports_every_symbol():
    L = asp.lib()
    for name in header_symbols():
        assert hasattr(L, name), name


def test_binding_declares_every_signature():
    """Every export has its argument types declared: ctypes would otherwise pass
    pointers as 32-bit ints."""
    L = asp.lib()
    for name in asp.EXPORTS:
        assert getattr(L, name).argtypes is not None, name


def test_default_options():
    opt = asp.default_options()
    assert opt.struct_size == ctypes.sizeof(asp.Options)
    assert (opt.max_iter, opt.max_active, opt.lm_max_iter, opt.init_mode) == (1000, 5, 100, 0)
    assert (opt.window_sigmas, opt.lm_mu0, opt.lm_tol, opt.psf_lobe_frac) == (5.0, 1e-3, 1e-5, 0.35)


def test_struct_layouts_match_header(tmp_path):
    """sizeof/offsetof from the C header (compiled by gcc) vs the ctypes mirrors."""
    structs = {"asp_options": asp.Options, "asp_component": asp.Component,
               "asp_fit_report": asp.FitReport, "asp_run_report": asp.RunReport,
               "asp_gauss": asp.Gauss, "asp_fit2004_report": asp.Fit2004Report}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "asp.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


@pytest.mark.parametrize("kw", [dict(gain=0.0), dict(gain=1.5), dict(threshold=-1.0),
                                dict(H=0), dict(max_active=0), dict(max_active=17),
                                dict(lm_max_iter=0), dict(psf_lobe_frac=1.0)])
def test_invalid_arguments_return_before_any_device_call(kw):
    H = kw.pop("H", 8)
    gain = kw.pop("gain", 0.1)
    thr = kw.pop("threshold", 0.0)
    opt = asp.default_options(**kw)
    img = np.zeros((8, 8), np.float32)
    ctx = ctypes.c_void_p()
    rc = asp.lib().asp_create(img.ctypes.data, H, 8, img.ctypes.data, 8, 8, gain, thr,
                              ctypes.byref(opt), ctypes.byref(ctx))
    assert rc == asp.ASP_ERR_INVALID_ARG and not ctx.value


def test_bad_struct_size_rejected():
    opt = asp.default_options()
    opt.struct_size = 12
    img = np.zeros((8, 8), np.float32)
    ctx = ctypes.c_void_p()
    rc = asp.lib().asp_create(img.ctypes.data, 8, 8, img.ctypes.data, 8, 8, 0.1, 0.0,
                              ctypes.byref(opt), ctypes.byref(ctx))
    assert rc == asp.ASP_ERR_INVALID_ARG


def test_null_context_calls():
    L = asp.lib()
    assert L.asp_find_peak(None, None, None) == asp.ASP_ERR_INVALID_ARG
    assert L.asp_run(None, 1, None) == asp.ASP_ERR_INVALID_ARG
    assert L.asp_last_error(None) == b"null context"
    assert L.asp_step_2004(None, None) == asp.ASP_ERR_INVALID_ARG
    assert L.asp_run_2004(None, 1, None) == asp.ASP_ERR_INVALID_ARG
    assert L.asp_model_image(None, None) == asp.ASP_ERR_INVALID_ARG
    assert L.asp_state_size(None, None) == asp.ASP_ERR_INVALID_ARG
    assert L.asp_save_state(None, None, 0, None) == asp.ASP_ERR_INVALID_ARG
    assert L.asp_load_state(None, None, 0) == asp.ASP_ERR_INVALID_ARG
    assert L.asp_residual_sumsq_tracked(None, None) == asp.ASP_ERR_INVALID_ARG
