"""Lockstep parity of the HIP minor cycle against the FP64 oracle, and the
invariants that hold at any size (flux conservation, the residual's plain
definition) on free runs."""
import numpy as np
import pytest

import oracle
import skygen
from parity import Lockstep

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")


def make_ctx(f, **kw):
    opts = dict(max_iter=f.max_iter, max_active=f.max_active)
    opts.update(kw)
    return asp.Context(f.dirty, f.psf, f.gain, f.threshold, **opts)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lockstep_c128(seed):
    f = skygen.make_c128(seed)
    print("lockstep c128 seed", seed, flush=True)
    ctx = make_ctx(f)
    ls = Lockstep(ctx, f)
    n_strict = 0
    for it in range(60):
        rec = ls.step()
        if rec is None:
            break
        strict = rec["gpu_conv"] and rec["orc_conv"]
        ls.check(rec, strict=strict)
        n_strict += strict
    assert n_strict >= 50
    ctx.close()


def test_lockstep_k1_isolated_gaussian():
    """K_max = 1 (Eq. 4 literally) on a noise-free isolated Gaussian: exact recovery."""
    img = skygen.isolated_gaussian(96, 96, 1.3, 40.3, 37.8, 2.7).astype(np.float32)
    psf = skygen.gaussian_psf(33, 3.0).astype(np.float32)
    f = skygen.Field("iso", img, psf, 1.0, 0.0, 4, 1, np.zeros((0, 3)), np.zeros((0, 4)), 0.0)
    ctx = make_ctx(f)
    ls = Lockstep(ctx, f)
    rec = ls.step()
    ls.check(rec)
    a, x, y, s = rec["gpu_theta"][0]
    assert abs(a - 1.3) < 1e-4 and abs(x - 40.3) < 1e-4 and abs(y - 37.8) < 1e-4
    assert abs(s - 2.7) < 1e-4
    ctx.close()


def gpu_model_sum(comps, H, W, ws=5.0):
    total = 0.0
    for a, x, y, s in comps:
        r0, r1, c0, c1 = oracle.box(x, y, oracle.halfwidth(s, ws), H, W)
        total += skygen.isolated_gaussian(H, W, a, x, y, s)[r0:r1 + 1, c0:c1 + 1].sum()
    return total


def test_free_run_c128_invariants():
    f = skygen.make_c128(0)
    ctx = make_ctx(f)
    rc, rep = ctx.run(f.max_iter)
    assert rc in (asp.ASP_OK, asp.ASP_STOP_THRESHOLD, asp.ASP_STOP_MAXITER)
    R = ctx.residual().astype(np.float64)
    comps = ctx.components_raw()
    H, W = f.shape
    # flux: sum(dirty) = sum(R) + sum of every component on its window
    total = f.dirty.astype(np.float64).sum()
    assert abs(total - R.sum() - gpu_model_sum(comps, H, W)) <= 1e-5 * np.abs(f.dirty).sum()
    # the residual from its definition, dirty - sum_j G_j on W_j
    ab, wb = ctx.psf_gauss()
    orc = oracle.Oracle(f.dirty, alpha_b=ab, omega_b=wb, max_iter=len(comps) + 1)
    orc.load_state(f.dirty, comps, len(comps))
    scratch = orc.residual_from_scratch()
    assert np.abs(scratch - R).max() <= 1e-4 * np.abs(f.dirty).max()
    assert np.sqrt((R ** 2).mean()) < 0.5 * np.sqrt((f.dirty.astype(float) ** 2).mean())
    ctx.close()


def test_run_matches_step_api():
    """asp_run and the step API take the same path: identical state after N."""
    f = skygen.make_c128(1)
    a = make_ctx(f)
    b = make_ctx(f)
    a.run(25)
    for _ in range(25):
        b.step()
    assert np.array_equal(a.residual(), b.residual())
    assert np.array_equal(a.components_raw(), b.components_raw())
    a.close()
    b.close()


def test_stop_threshold_on_device():
    img = skygen.isolated_gaussian(32, 32, 1.0, 16.0, 16.0, 1.3).astype(np.float32)
    psf = skygen.gaussian_psf(33, 1.3 * skygen.FWHM_PER_SIGMA).astype(np.float32)
    ctx = asp.Context(img, psf, 0.5, 0.3, max_iter=50, max_active=1)
    rc, rep = ctx.run(50)
    assert rc == asp.ASP_STOP_THRESHOLD
    assert rep["iterations"] == 2       # 1.0 -> 0.5 -> 0.25 < 0.3
    rc, rep = ctx.run(5)
    assert rc == asp.ASP_STOP_THRESHOLD and rep["iterations"] == 0
    ctx.close()
    ctx = asp.Context(img, psf, 0.5, 0.0, max_iter=3, max_active=1)
    rc, rep = ctx.run(10)
    assert rc == asp.ASP_STOP_MAXITER and rep["iterations"] == 3
    ctx.close()


def test_lockstep_c1024_sampled():
    f = skygen.make_c1024(1000)
    print("lockstep c1024", flush=True)
    ctx = make_ctx(f)
    ls = Lockstep(ctx, f)
    for it in range(6):
        rec = ls.step()
        ls.check(rec, strict=rec["gpu_conv"] and rec["orc_conv"])
    rc, rep = ctx.run(300)
    assert rc == asp.ASP_OK
    for it in range(6):
        rec = ls.step()
        ls.check(rec, strict=rec["gpu_conv"] and rec["orc_conv"])
    ctx.close()


@pytest.mark.parametrize("name,target,steps", [("c1024", 4000, 4), ("c1024", 4990, 4),
                                               ("c4096", 12000, 3)])
def test_lockstep_late_iterations(name, target, steps):
    """Lockstep deep into the configured runs (the 1024^2 field's 5000
    iterations, the 4096^2 field's 20000): the device runs to the target
    iteration on its own, then the oracle is loaded with its state and both
    step together."""
    f = skygen.make_c1024(1000) if name == "c1024" else skygen.make_c4096(4096)
    print("lockstep", name, "from iteration", target, flush=True)
    ctx = make_ctx(f)
    rc, rep = ctx.run(target)
    assert rc == asp.ASP_OK and rep["iterations"] == target
    ls = Lockstep(ctx, f)
    n_strict = 0
    for it in range(steps):
        rec = ls.step()
        assert rec is not None
        strict = rec["gpu_conv"] and rec["orc_conv"]
        print(f"k={rec['k']} members {rec['members']} conv {rec['gpu_conv']}/{rec['orc_conv']} "
              f"resid {rec['resid_err']:.3g} cond {rec['cond']:.3g}", flush=True)
        ls.check(rec, strict=strict)
        n_strict += strict
    assert n_strict >= 1
    ctx.close()
