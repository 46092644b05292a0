"""One LM trial's reduced sums on the device against the FP64 oracle
(Sect. 3, Eq. 4): asp_eval_trial runs the fit kernel's own evaluation path --
the register path for one and two members, the LDS path above, a single
work-group for small unions of windows and the whole grid for large ones --
and returns J^T J, J^T r, F, chi2 and |U|; the oracle's fit_eval computes
them in FP64 from the same residual and parameters.

The kernel forms D, M and r in FP64 and rounds J and r to FP32 for the Gram
sums (FP64 accumulation for one or two members, FP32 tile sums with Kahan
compensation across tiles above), so its Gram entries carry a relative error
of the order of the FP32 unit roundoff: the tolerance is 1e-6 of the entry's
Cauchy-Schwarz scale, |dH_ik| <= 1e-6 sqrt(H_ii H_kk) and |dg_i| <= 1e-6
sqrt(H_ii chi2).  F and chi2 are FP64 sums: 1e-9 relative."""
import numpy as np
import pytest

import oracle
import skygen

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")


def field(n, seed):
    rng = np.random.default_rng(seed)
    img = rng.normal(0.0, 0.05, size=(n, n))
    for _ in range(12):
        x, y = rng.uniform(0.2 * n, 0.8 * n, size=2)
        s = rng.uniform(2.0, n / 16)
        img += rng.uniform(0.2, 1.0) * skygen.isolated_gaussian(n, n, 1.0, x, y, s)
    return img.astype(np.float32)


def members(m, n, seed, s_lo, s_hi):
    """m members around the image centre with overlapping windows, widths away
    from the window-size steps; stored = perturbed copies (row 0 unused)."""
    rng = np.random.default_rng(seed)
    c = n / 2.0
    th = np.zeros((m, 4))
    for j in range(m):
        s = rng.uniform(s_lo, s_hi)
        s = (np.floor(5 * s) + 0.5) / 5.0          # 5 s half-way between integers
        th[j] = [rng.uniform(0.2, 1.0), c + rng.uniform(-3, 3) * s_hi + 0.13,
                 c + rng.uniform(-3, 3) * s_hi + 0.29, s]
    st = th.copy()
    st[:, 0] *= rng.uniform(0.8, 1.2, size=m)
    st[:, 1:3] += rng.uniform(-0.3, 0.3, size=(m, 2))
    st[:, 3] *= rng.uniform(0.95, 1.05, size=m)
    st[:, 3] = (np.floor(5 * st[:, 3]) + 0.5) / 5.0
    st[0] = 0.0
    return th, st


CASES = {
    # name: (image size, members, width range) -- small unions: one work-group
    "m1_small": (256, 1, 1.5, 3.0),
    "m2_small": (256, 2, 1.5, 3.0),
    "m5_small": (256, 5, 1.5, 4.0),
    "m10_small": (256, 10, 1.5, 4.0),
    "m16_small": (256, 16, 1.2, 3.0),
    # large unions: shared by the whole grid
    "m1_large": (1024, 1, 30.0, 40.0),
    "m2_large": (1024, 2, 20.0, 35.0),
    "m5_large": (1024, 5, 10.0, 25.0),
    "m10_large": (1024, 10, 8.0, 20.0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_trial_sums_match_oracle(case):
    n, m, s_lo, s_hi = CASES[case]
    dirty = field(n, 11 + n)
    psf = skygen.gaussian_psf(31, 3.0).astype(np.float32)
    ctx = asp.Context(dirty, psf, 0.1, 0.0, max_iter=10, max_active=16)
    th, st = members(m, n, 5 + m, s_lo, s_hi)
    got = ctx.eval_trial(th, st)
    ab, wb = ctx.psf_gauss()
    o = oracle.Oracle(ctx.residual(), gain=0.1, max_iter=10, max_active=16, alpha_b=ab, omega_b=wb)
    ref = o.fit_eval(th, st)
    ctx.close()
    H, g = ref["H"], ref["g"]
    d = np.sqrt(np.maximum(np.diag(H), 0.0))
    scale_h = np.outer(d, d)
    scale_g = d * np.sqrt(ref["chi2"])
    eh = np.abs(got["H"] - H) / np.maximum(scale_h, 1e-300)
    eg = np.abs(got["g"] - g) / np.maximum(scale_g, 1e-300)
    eF = abs(got["F"] - ref["F"]) / (abs(ref["F"]) + ref["chi2"])
    ec = abs(got["chi2"] - ref["chi2"]) / ref["chi2"]
    print(f"{case}: |U| {ref['npx']}, errors H {eh.max():.3g} g {eg.max():.3g} "
          f"F {eF:.3g} chi2 {ec:.3g}", flush=True)
    assert got["npx"] == ref["npx"]
    assert eh.max() <= 1e-6 and eg.max() <= 1e-6
    assert eF <= 1e-9 and ec <= 1e-9


def test_eval_trial_rejects_bad_arguments():
    dirty = field(64, 3)
    psf = skygen.gaussian_psf(15, 3.0).astype(np.float32)
    ctx = asp.Context(dirty, psf, 0.1, 0.0, max_iter=10, max_active=16)
    with pytest.raises(asp.AspError):
        ctx.eval_trial(np.zeros((17, 4)) + 1.0)
    with pytest.raises(asp.AspError):
        ctx.eval_trial([[1.0, 30.0, 30.0, 0.0]])
    with pytest.raises(asp.AspError):
        ctx.eval_trial([[1.0, np.nan, 30.0, 2.0]])
    # the context is unchanged and still runs
    rc, rep = ctx.run(3)
    assert rep["iterations"] == 3
    ctx.close()
