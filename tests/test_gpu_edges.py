"""Edge cases of the HIP minor cycle: invalid images, the stop and capacity
rules, degenerate image shapes, the largest active set, call-order errors,
and lockstep parity at the full 4096 x 4096 size."""
import numpy as np
import pytest

import oracle
import skygen
from parity import COND_MAX, scaled_cond, Lockstep, RESID_TOL, param_errors

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")


def gauss_psf(n=9, fwhm=2.5):
    return skygen.gaussian_psf(n, fwhm).astype(np.float32)


@pytest.mark.parametrize("where", ["dirty_nan", "dirty_inf", "psf_nan"])
def test_nonfinite_input_is_rejected(where):
    dirty = np.zeros((32, 32), np.float32)
    dirty[10, 10] = 1.0
    psf = gauss_psf()
    if where == "dirty_nan":
        dirty[3, 4] = np.nan
    elif where == "dirty_inf":
        dirty[31, 31] = np.inf
    else:
        psf[0, 0] = np.nan
    with pytest.raises(asp.AspError) as e:
        asp.Context(dirty, psf, 0.1, 0.0)
    assert e.value.status == asp.ASP_ERR_NONFINITE


def test_zero_image_stops_at_once():
    ctx = asp.Context(np.zeros((64, 64), np.float32), gauss_psf(), 0.1, 1e-3, max_iter=10)
    rc, rep = ctx.run(10)
    assert rc == asp.ASP_STOP_THRESHOLD and rep["iterations"] == 0
    assert ctx.counts() == (0, 0)
    ctx.close()


def test_capacity_is_an_error_after_the_last_slot():
    f = skygen.make_c128(4)
    ctx = asp.Context(f.dirty, f.psf, f.gain, 0.0, max_iter=50, capacity=3)
    with pytest.raises(asp.AspError) as e:
        ctx.run(10)
    assert e.value.status == asp.ASP_ERR_CAPACITY
    k, L = ctx.counts()
    assert L == 3 and k >= 3
    ctx.close()


def test_call_order_is_enforced():
    f = skygen.make_c128(5)
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold)
    with pytest.raises(asp.AspError) as e:
        ctx.update_residual()
    assert e.value.status == asp.ASP_ERR_STATE
    with pytest.raises(asp.AspError) as e:
        ctx.fit_active_set(0)
    assert e.value.status == asp.ASP_ERR_STATE
    rc, idx, val = ctx.find_peak()
    with pytest.raises(asp.AspError):
        ctx.run(1)                      # inside a step-API sequence
    ctx.fit_active_set(idx)
    ctx.update_residual()
    ctx.close()


@pytest.mark.parametrize("shape", [(1, 1), (2, 2), (3, 5), (7, 1), (1, 9)])
def test_degenerate_shapes_in_lockstep(shape):
    """Images smaller than a window: every window is clipped to the image."""
    H, W = shape
    dirty = np.zeros(shape, np.float32)
    dirty[H // 2, W // 2] = 1.0
    if H * W > 1:
        dirty.flat[0] = -0.3
    psf = gauss_psf()
    ctx = asp.Context(dirty, psf, 0.3, 0.0, max_iter=6)
    ab, wb = ctx.psf_gauss()
    orc = oracle.Oracle(dirty, gain=0.3, threshold=0.0, max_iter=6, max_active=5,
                        alpha_b=ab, omega_b=wb)
    for it in range(6):
        R0, comps0, k0 = ctx.residual(), ctx.components_raw(), ctx.counts()[0]
        rc, idx, val = ctx.find_peak()
        rc, rep = ctx.fit_active_set(idx)
        ctx.update_residual()
        orc.load_state(R0, comps0, k0)
        orep = orc.step()
        assert orep["idx"] == idx and orep["members"] == rep["members"], (shape, it)
        R1 = ctx.residual().astype(np.float64)
        assert np.abs(R1 - orc.R).max() <= RESID_TOL, (shape, it)
    ctx.close()


def crowded_field(seed=11, n=64, count=40):
    """Overlapping same-sign Gaussians in the middle of a small image: the
    active set fills up to its maximum."""
    rng = np.random.default_rng(seed)
    img = np.zeros((n, n))
    for _ in range(count):
        x, y = rng.uniform(24, 40, size=2)
        s = rng.uniform(1.5, 5.0)
        img += rng.uniform(0.2, 1.0) * skygen.isolated_gaussian(n, n, 1.0, x, y, s)
    return img.astype(np.float32)


def test_lockstep_largest_active_set():
    """K_max = 16 (n = 64 parameters, 2145 Gram entries per pixel): the
    work-group Gram path and the work-group Cholesky solve, in lockstep."""
    dirty = crowded_field()
    psf = gauss_psf(15, 3.0)
    ctx = asp.Context(dirty, psf, 0.3, 0.0, max_iter=200, max_active=16)
    ab, wb = ctx.psf_gauss()
    orc = oracle.Oracle(dirty, gain=0.3, threshold=0.0, max_iter=200, max_active=16,
                        alpha_b=ab, omega_b=wb, cap=201)
    peak = float(np.abs(dirty).max())
    ctx.run(40)                         # build up a crowd of components
    m_max, n_strict = 0, 0
    for it in range(40):
        if m_max >= 8 and n_strict >= 6:
            break
        R0, comps0, k0 = ctx.residual(), ctx.components_raw(), ctx.counts()[0]
        rc, idx, val = ctx.find_peak()
        rc, rep = ctx.fit_active_set(idx)
        ctx.update_residual()
        orc.load_state(R0, comps0, k0)
        orep = orc.step(want_hess=True)
        assert orep["idx"] == idx and orep["members"] == rep["members"], it
        m_max = max(m_max, rep["n_active"])
        cond = scaled_cond(orep["hess"])
        R1 = ctx.residual().astype(np.float64)
        err = float(np.abs(R1 - orc.R).max())
        pe = param_errors(rep["theta"], orep["theta"]).max()
        print(f"iteration {k0}: m {rep['n_active']} converged {rep['converged']}/"
              f"{orep['converged']} trials {rep['lm_iters']}/{orep['lm_iters']} added "
              f"{rep['added']}/{orep['added']} param err/tol {pe:.3g} resid err/tol "
              f"{err / (RESID_TOL * peak):.3g} cond {cond:.3g}", flush=True)
        assert rep["added"] == orep["added"], it
        if rep["converged"] and orep["converged"]:
            assert err <= RESID_TOL * peak, it
            # an ill-conditioned joint fit determines the members' sum, not
            # each member: then the residual alone is compared
            assert pe <= 1.0 or cond > COND_MAX, it
            n_strict += 1
        else:
            # a fit that used its whole budget on both sides stops at different
            # points of an ill-conditioned path: the residual must still be
            # the dirty image minus the committed list
            orc.load_state(dirty, ctx.components_raw(), k0 + 1)
            want = orc.residual_from_scratch()
            assert np.abs(R1 - want).max() <= RESID_TOL * peak, it
    print("largest active set", m_max, "strict", n_strict, flush=True)
    assert m_max >= 8 and n_strict >= 6
    ctx.close()


def test_lockstep_c4096_sampled():
    """The 4096 x 4096 field in the configuration the benchmark times: lockstep
    at the first iterations and after 200 device-resident ones."""
    f = skygen.make_c4096(4096)
    print("lockstep c4096", flush=True)
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter,
                      max_active=f.max_active)
    ls = Lockstep(ctx, f)
    for it in range(3):
        rec = ls.step()
        ls.check(rec, strict=rec["gpu_conv"] and rec["orc_conv"])
    rc, rep = ctx.run(200)
    assert rc == asp.ASP_OK
    for it in range(3):
        rec = ls.step()
        ls.check(rec, strict=rec["gpu_conv"] and rec["orc_conv"])
    ctx.close()
