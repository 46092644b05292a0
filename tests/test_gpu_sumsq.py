"""The tracked sum of R^2 (asp_residual_sumsq_tracked, for a noise-level stop
rule, Sect. 2 step 4): windowed deltas of the updates on a base that a full
pass re-sets whenever the whole residual changes.  Compared with the full
pass on the device and with the FP64 sum of the copied residual, through plain
steps, runs, the smoothing method with the incremental peak search, exact-PSF
refreshes, the Asp-Clean2004 iteration, a state load and a batch."""
import numpy as np
import pytest

import skygen

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")

# Each update adds per pixel the FP64 difference of two exact squares of FP32
# values, rounded once, then sums in a fixed order: the error after n updates
# is about n * 2^-53 of the sums it went through, i.e. relative to the sum at
# the last re-base (the residual only shrinks after it), not to the current one.
REL = 1e-12


def host_sumsq(ctx):
    R = ctx.residual().astype(np.float64)
    return float(np.sum(R * R))


def check(ctx, what, base):
    """Tracked vs the host's FP64 sum, to REL of the sum at the last re-base
    (base); then the full pass re-bases and the tracked read equals it.
    Returns the new base."""
    tracked = ctx.residual_sumsq(tracked=True)
    want = host_sumsq(ctx)
    print(f"{what}: tracked {tracked!r} host {want!r} error/base "
          f"{abs(tracked - want) / base:.3g}", flush=True)
    assert abs(tracked - want) <= REL * base, what
    full = ctx.residual_sumsq()             # re-bases
    assert abs(full - want) <= REL * want, what
    assert ctx.residual_sumsq(tracked=True) == full, what
    return full


def dirty_sumsq(f):
    d = np.asarray(f.dirty, np.float64)
    return float(np.sum(d * d))


def make(f, **kw):
    opts = {"max_iter": f.max_iter, "max_active": f.max_active}
    opts.update(kw)
    return asp.Context(f.dirty, f.psf, f.gain, f.threshold, **opts)


@pytest.mark.parametrize("kw", [{}, {"init_mode": 2, "peak_tiles": 1}, {"refresh_every": 10}],
                         ids=["simple", "smoothing+tiles", "refresh"])
def test_tracked_sum_follows_the_updates(kw):
    f = skygen.make_evla(256, 11, 60, 6, 16.0, 400, 5, psf_crop=128)
    ctx = make(f, **kw)
    base = dirty_sumsq(f)
    # 40 iterations on the base set at create: the deltas alone
    ctx.run(40)
    tracked = ctx.residual_sumsq(tracked=True)
    want = host_sumsq(ctx)
    assert abs(tracked - want) <= REL * base
    base = check(ctx, "run 40", base)
    for _ in range(5):                      # the step sequence of the minor cycle
        rc, idx, _ = ctx.find_peak()
        assert rc == asp.ASP_OK
        ctx.fit_active_set(idx)
        ctx.update_residual()
    base = check(ctx, "steps", base)
    ctx.run(200)
    check(ctx, "run 200", base)
    ctx.close()


def test_tracked_sum_at_4096():
    f = skygen.make_c4096(4096)
    ctx = make(f, max_iter=400)
    ctx.run(300)
    check(ctx, "c4096 after 300 iterations", dirty_sumsq(f))
    ctx.close()


def test_tracked_sum_through_2004_and_a_load():
    f = skygen.make_evla(128, 7, 40, 4, 10.0, 200, 1, psf_crop=128)
    a = make(f)
    a.run(10)
    a.run_2004(2)                           # re-bases after each update
    base = check(a, "2004", a.residual_sumsq())
    a.run(10)
    blob = a.save_state()
    a.residual_sumsq()                      # re-base where the load re-bases
    a.run(10)
    b = make(f)
    b.load_state(blob)
    b.run(10)
    # the same base and the same deltas in the same slots: bit for bit
    assert b.residual_sumsq(tracked=True) == a.residual_sumsq(tracked=True)
    check(b, "loaded", base)
    a.close()
    b.close()


def test_tracked_sum_in_a_batch():
    fields = [skygen.make_c128(s) for s in (0, 1, 2)] + [skygen.make_c1024(1000)]
    b = asp.Batch([(f.dirty, f.psf, f.gain, f.threshold) for f in fields], max_iter=200)
    b.run(150)
    for i in range(len(fields)):
        check(b.field(i), f"batch field {i}", dirty_sumsq(fields[i]))
    b.close()


@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (7, 1), (1, 9)])
def test_tracked_sum_on_degenerate_shapes(shape):
    """Images smaller than a window: every update window is clipped."""
    H, W = shape
    dirty = np.zeros(shape, np.float32)
    dirty[H // 2, W // 2] = 1.0
    if H * W > 1:
        dirty.flat[0] = -0.3
    psf = skygen.gaussian_psf(33, 3.0).astype(np.float32)
    ctx = asp.Context(dirty, psf, 0.3, 0.0, max_iter=6)
    ctx.run(6)
    check(ctx, f"shape {shape}", float(np.sum(dirty.astype(np.float64) ** 2)))
    ctx.close()
