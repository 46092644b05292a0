"""The residual update at the end of the fit kernel (asp_run's default) against
its own launch (update_launch=1, as asp_update_residual runs it): every pixel
is rewritten by one work-group with the same arithmetic in the same order, so
the two runs must agree bit for bit, including the stale-tile marking of the
incremental peak search and of the smoothed images."""
import numpy as np
import pytest

import skygen

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")


def make(f, **kw):
    opts = {"max_iter": 400, "max_active": f.max_active}
    opts.update(kw)
    return asp.Context(f.dirty, f.psf, f.gain, f.threshold, **opts)


@pytest.mark.parametrize("kw", [{}, {"init_mode": 2, "peak_tiles": 1}, {"refresh_every": 20}],
                         ids=["simple", "smoothing+tiles", "refresh"])
def test_fused_update_equals_its_own_launch(kw):
    f = skygen.make_evla(256, 11, 60, 6, 16.0, 400, 5, psf_crop=128)
    a = make(f, update_launch=0, **kw)
    b = make(f, update_launch=1, **kw)
    a.kernel_timing(True)
    b.kernel_timing(True)
    ra = a.run(120)
    rb = b.run(120)
    assert ra == rb
    assert np.array_equal(a.residual(), b.residual())
    assert np.array_equal(a.components_raw(), b.components_raw())
    ka, kb = a.kernel_times(), b.kernel_times()
    assert ka["update"][1] == 0 and kb["update"][1] == 120
    # the tracked sum of R^2 follows both (the slots differ, the sum agrees)
    for c in (a, b):
        want = float(np.sum(c.residual().astype(np.float64) ** 2))
        assert abs(c.residual_sumsq(tracked=True) - want) <= 1e-12 * float(
            np.sum(f.dirty.astype(np.float64) ** 2))
    a.close()
    b.close()


def test_fused_update_c4096():
    f = skygen.make_c4096(4096)
    a = make(f, update_launch=0)
    b = make(f, update_launch=1)
    ra = a.run(60)
    rb = b.run(60)
    assert ra == rb
    assert np.array_equal(a.residual(), b.residual())
    assert np.array_equal(a.components_raw(), b.components_raw())
    a.close()
    b.close()


def test_update_launch_option_is_checked():
    f = skygen.make_c128(0)
    with pytest.raises(asp.AspError):
        make(f, update_launch=2)
    with pytest.raises(asp.AspError):
        make(f, reserved=1)
