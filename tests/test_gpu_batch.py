"""Batched fields on the GPU: one persistent, graph-captured launch over
fields of uneven size.  Each field is checked against the FP64 oracle in
lockstep (one iteration per launch), and free runs over several graph replays
against the invariants that hold at any size."""
import numpy as np
import pytest

import oracle
import skygen
from parity import param_errors, RESID_TOL

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")

SIZES = [512, 96, 192, 64, 128]


def small_fields(max_iter=400):
    return [skygen.make_batch_field(n, 7000 + i, max_iter) for i, n in enumerate(SIZES)]


def make_batch(fields, **kw):
    return asp.Batch([(f.dirty, f.psf, f.gain, f.threshold) for f in fields],
                     max_iter=fields[0].max_iter, max_active=5, **kw)


def batch_lockstep(fields, team, n_iter, min_strict, pre_iters=0):
    """One iteration per launch; each field's oracle is loaded with the field's
    pre-launch state and steps once.  Peak, members (from the device's report
    of the field's last fit), whether the new component joined, the committed
    list and the residual are compared.  pre_iters: batched iterations run
    first, without comparison."""
    b = make_batch(fields)
    b.config(team_size=team)
    if pre_iters:
        rep = b.run(pre_iters)
        assert rep["fields_failed"] == 0 and rep["iterations"] == pre_iters * len(fields)
    print("batch config", b.get_config(), [f.shape for f in fields], flush=True)
    ctxs = [b.field(i) for i in range(len(fields))]
    orcs = []
    for f, c in zip(fields, ctxs):
        ab, wb = c.psf_gauss()
        orcs.append(oracle.Oracle(f.dirty, gain=f.gain, threshold=f.threshold,
                                  max_iter=f.max_iter, max_active=5, alpha_b=ab, omega_b=wb,
                                  cap=f.max_iter + 1))
    n_strict = 0
    for it in range(n_iter):
        pre = [(c.residual(), c.components_raw(), c.counts()[0]) for c in ctxs]
        rep = b.run(1)
        assert rep["fields_failed"] == 0
        for i, (f, c, o) in enumerate(zip(fields, ctxs, orcs)):
            R0, comps0, k0 = pre[i]
            o.load_state(R0, comps0, k0)
            orep = o.step()
            k1, L1 = c.counts()
            assert k1 == k0 + 1, (i, k0, k1)
            last = c.last_fit()
            assert last["idx"] == orep["idx"], (i, it, last["idx"], orep["idx"])
            assert last["members"] == orep["members"], (i, it, last["members"], orep["members"])
            assert last["added"] == orep["added"], (i, it)
            comps1 = c.components_raw()
            assert comps1.shape == o.comps().shape, (i, it)
            strict = orep["converged"] and last["converged"]
            if strict:
                assert np.all(param_errors(last["theta"], orep["theta"]) <= 1.0), (i, it)
                assert np.all(param_errors(comps1, o.comps()) <= 1.0), (i, it)
            R1 = c.residual().astype(np.float64)
            peak = float(np.abs(f.dirty).max())
            assert np.abs(R1 - o.R).max() <= RESID_TOL * peak, (i, it)
            n_strict += strict
    assert n_strict >= min_strict
    b.close()


@pytest.mark.parametrize("team", [4, 8])
def test_batch_lockstep_per_field(team):
    batch_lockstep(small_fields(), team, 8, 30)


def test_batch_lockstep_large_fields():
    """Fields of the batched workload's larger sizes, 2048^2 and 1024^2 (and a
    256^2 one), with a team of 32 work-groups: shared peak scans, shared
    trials and shared updates on every field."""
    fields = [skygen.make_batch_field(n, 7100 + i, 400) for i, n in enumerate([2048, 1024, 256])]
    batch_lockstep(fields, 32, 4, 9)


def test_batch_lockstep_late_in_the_run():
    """The same comparison after 1500 batched iterations per field, on fields of
    2048^2, 1024^2 and 512^2 with a team of 16 work-groups."""
    fields = [skygen.make_batch_field(n, 7400 + i, 2000) for i, n in enumerate([2048, 1024, 512])]
    batch_lockstep(fields, 16, 3, 3, pre_iters=1500)


def test_batch_replays_keep_invariants():
    """Three replays of the captured launch (10 iterations per field each): every
    field advances by 30 iterations and its residual equals the dirty image
    minus its component list (evaluated by the oracle from scratch)."""
    fields = small_fields()
    b = make_batch(fields)
    b.config(team_size=8)
    for r in range(3):
        rep = b.run(10)
        assert rep["fields_failed"] == 0
        print("replay", r, rep, flush=True)
    for i, f in enumerate(fields):
        c = b.field(i)
        k, L = c.counts()
        comps = c.components_raw()
        # a new component of amplitude zero is not added
        assert k == 30 and L <= 30 and comps.shape[0] == L and np.all(comps[:, 0] != 0.0)
        ab, wb = c.psf_gauss()
        o = oracle.Oracle(f.dirty, gain=f.gain, threshold=f.threshold, max_iter=f.max_iter,
                          max_active=5, alpha_b=ab, omega_b=wb, cap=f.max_iter + 1)
        o.load_state(f.dirty, c.components_raw(), k)
        want = o.residual_from_scratch()
        got = c.residual().astype(np.float64)
        assert np.abs(got - want).max() <= RESID_TOL * float(np.abs(f.dirty).max()), i
    b.close()


def test_batch_autotune_picks_a_valid_config():
    fields = small_fields()
    b = make_batch(fields)
    cfg = b.autotune(2)
    print("autotuned", cfg, flush=True)
    grid = b.get_config()["grid"]
    assert (grid // 8) % cfg["team_size"] == 0
    assert cfg["solo_tiles"] in (4, 8, 16, 32) and cfg["min_tiles"] in (1, 2, 4)
    k = [b.field(i).counts()[0] for i in range(len(fields))]
    assert all(v == k[0] for v in k) and k[0] > 0
    b.close()


def test_batch_rejects_bad_team_size():
    fields = small_fields()[:2]
    b = make_batch(fields)
    with pytest.raises(asp.AspError):
        b.config(team_size=3)
    b.close()


def test_batch_leader_working_alone_for_seconds():
    """A 64 x 64 field with a team of 8: its leader scans, fits and updates
    alone (every trial is at most 16 tiles, under solo_tiles 32), so its
    followers get no command for the whole run, well past the 2 s bound of a
    wait.  Their waits restart on the leader's per-iteration heartbeat, so the
    field does not fail."""
    f = skygen.make_batch_field(64, 7300, 20000)
    b = asp.Batch([(f.dirty, f.psf, f.gain, 0.0)], max_iter=20000, max_active=5)
    b.config(team_size=8, solo_tiles=32)
    rep = b.run(12000)
    print("solo leader run", rep, flush=True)
    assert rep["fields_failed"] == 0
    k, L = b.field(0).counts()
    assert k == 12000
    assert rep["ms"] > 2500, "the run must outlast the 2 s bound of a wait"
    b.close()
