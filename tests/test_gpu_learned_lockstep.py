"""Lockstep parity of the learned start with the committed network
(paper_1606_07872_amd/proposal_weights.npy) on the 1024^2 and 4096^2
EVLA-like fields.  The device runs its minor cycle in learned mode; at sampled
iterations it fits one iteration from its own proposal, and the oracle, loaded
with the device's pre-step state, fits from that same proposal (Sect. 3 with
the proposal as the initial values of the new component): same peak, same
members, the same choice between the proposal and the simple values, the same
fallback, and parameters and residual within the lockstep tolerances."""
import os

import numpy as np
import pytest

import skygen
from parity import Lockstep

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")

WEIGHTS = os.path.join(os.path.dirname(asp.__file__), "proposal_weights.npy")

# field: (generator, [(iteration to run to, lockstep iterations from there)])
CASES = {
    "c1024": (lambda: skygen.make_c1024(1000), [(0, 6), (1000, 4), (3000, 4)]),
    "c4096": (lambda: skygen.make_c4096(4096), [(0, 3), (2000, 3)]),
}


@pytest.mark.parametrize("name", list(CASES))
def test_learned_lockstep_with_committed_weights(name):
    make, samples = CASES[name]
    f = make()
    w = np.load(WEIGHTS)
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter,
                      max_active=f.max_active)
    ctx.set_mlp(w)
    ctx.set_init_mode(1)
    ls = Lockstep(ctx, f)
    n_prop = n_strict = 0
    for target, n_steps in samples:
        k, _ = ctx.counts()
        if target > k:
            rc, rep = ctx.run(target - k)
            assert rep["iterations"] == target - k
        for _ in range(n_steps):
            rec = ls.step(learned=True)
            assert rec is not None
            strict = rec["gpu_conv"] and rec["orc_conv"]
            print(f"{name} k={rec['k']}: members {rec['members']} proposal {rec['prop']} "
                  f"fallback {rec['fallback']}/{rec['orc_fallback']} conv {rec['gpu_conv']}/"
                  f"{rec['orc_conv']} resid {rec['resid_err']:.3g} cond {rec['cond']:.3g}",
                  flush=True)
            ls.check(rec, strict=strict)
            if strict:
                assert rec["fallback"] == rec["orc_fallback"], rec
                n_strict += 1
            n_prop += rec["prop"]
    ctx.close()
    assert n_prop >= 1
    assert n_strict >= len(ls.records) // 2
