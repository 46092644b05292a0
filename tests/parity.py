"""Shared helpers of the GPU parity tests: the lockstep protocol.

Lockstep: the GPU advances one iteration; the oracle is loaded with the GPU's
pre-step state (residual converted exactly from FP32 to FP64, the FP64
component list, the iteration count, the GPU's alpha_b/omega_b) and steps
once.  Then:
  * the peak index and the active-set members (in order) must be equal,
  * every member's a and s must agree to 1e-3 relative and x, y to
    1e-3 * max(1, s) pixels,
  * the residuals must agree to 1e-4 * max|dirty|,
  * both sides must agree on whether the new component joined the list, and
    the committed lists (old members moved by the loop gain toward their
    refits, the new component) must agree to the parameter tolerance.
"""
import numpy as np

import oracle

PARAM_RTOL = 1e-3
RESID_TOL = 1e-4
# Several correct results: when the fit's J^T J (scaled to unit diagonal) has a
# condition number above this, its members are not individually determined
# and only their sum -- the residual -- is compared.
COND_MAX = 1e8


def scaled_cond(H) -> float:
    """Condition number of J^T J scaled to unit diagonal (unit-free)."""
    H = np.asarray(H, dtype=np.float64)
    d = np.sqrt(np.maximum(np.diag(H), 1e-300))
    return float(np.linalg.cond(H / np.outer(d, d)))


def param_errors(gpu_theta, orc_theta):
    """Per-member error ratios (value / allowed) for a, x, y, s."""
    g = np.asarray(gpu_theta, dtype=np.float64).reshape(-1, 4)
    o = np.asarray(orc_theta, dtype=np.float64).reshape(-1, 4)
    out = []
    for (ga, gx, gy, gs), (oa, ox, oy, os_) in zip(g, o):
        ra = abs(ga - oa) / (PARAM_RTOL * max(abs(oa), 1e-30))
        rs = abs(gs - os_) / (PARAM_RTOL * os_)
        pos = PARAM_RTOL * max(1.0, os_)
        out.append((ra, abs(gx - ox) / pos, abs(gy - oy) / pos, rs))
    return np.array(out)


class Lockstep:
    def __init__(self, ctx, field, **orc_kw):
        self.ctx = ctx
        self.f = field
        ab, wb = ctx.psf_gauss()
        self.orc = oracle.Oracle(field.dirty, gain=field.gain, threshold=field.threshold,
                                 max_iter=field.max_iter, max_active=field.max_active,
                                 alpha_b=ab, omega_b=wb, cap=field.max_iter + 1, **orc_kw)
        self.peak = float(np.abs(field.dirty).max())
        self.records = []

    def step(self, init=None, learned=False):
        """One lockstep iteration.  With `learned` the context is in learned
        mode: the device fits from its network's proposal first, and the
        oracle then fits from that same proposal."""
        ctx, orc = self.ctx, self.orc
        R0 = ctx.residual()
        comps0 = ctx.components_raw()
        k0, _ = ctx.counts()
        rc, idx, val = ctx.find_peak()
        orc.load_state(R0, comps0, k0)
        if rc != 0:
            orep = orc.step(init=init, want_hess=True)
            assert orep["status"] == rc, (rc, orep["status"])
            return None
        if learned:
            rc, rep = ctx.fit_active_set(idx)
            assert rep["init_source"] == 2, rep["init_source"]
            orep = orc.step(init=rep["init"], want_hess=True)
        else:
            orep = orc.step(init=init, want_hess=True)
            rc, rep = ctx.fit_active_set(idx, init=init)
        ctx.update_residual()
        R1 = ctx.residual().astype(np.float64)
        rec = {"k": k0, "idx": idx, "orc_idx": orep["idx"], "members": rep["members"],
               "orc_members": orep["members"], "gpu_conv": rep["converged"],
               "orc_conv": orep["converged"], "gpu_theta": rep["theta"],
               "orc_theta": orep["theta"], "resid_err": float(np.abs(R1 - orc.R).max()),
               "gpu_trials": rep["lm_iters"], "orc_trials": orep["lm_iters"],
               "added": rep["added"], "orc_added": orep["added"],
               "prop": rep["start_from_proposal"], "orc_prop": orep["start_from_proposal"],
               "fallback": rep["used_fallback"], "orc_fallback": orep["used_fallback"],
               "cond": scaled_cond(orep["hess"]) if "hess" in orep else 0.0}
        if rec["members"] == rec["orc_members"]:
            rec["param_err"] = param_errors(rep["theta"], orep["theta"])
        comps1, ocomps = ctx.components_raw(), orc.comps()
        rec["n_comps"], rec["orc_n_comps"] = comps1.shape[0], ocomps.shape[0]
        if comps1.shape == ocomps.shape:
            # the members this step changed (and the new one): the others are
            # loaded from the same list and must be identical
            touched = [j for j in rep["members"][1:]] + list(range(comps0.shape[0], comps1.shape[0]))
            rec["comp_err"] = param_errors(comps1[touched], ocomps[touched]) if touched else \
                np.zeros((0, 4))
            keep = np.ones(comps1.shape[0], bool)
            keep[touched] = False
            rec["untouched_equal"] = bool(np.array_equal(comps1[keep], ocomps[keep]))
        self.records.append(rec)
        return rec

    def check(self, rec, strict=True):
        assert rec["idx"] == rec["orc_idx"], rec
        assert rec["members"] == rec["orc_members"], rec
        assert rec["resid_err"] <= RESID_TOL * self.peak, (rec["resid_err"], rec["k"])
        assert rec["added"] == rec["orc_added"], rec
        assert rec["prop"] == rec["orc_prop"], rec
        assert rec["n_comps"] == rec["orc_n_comps"], rec
        assert rec["untouched_equal"], rec
        if strict and rec["cond"] <= COND_MAX:
            assert rec["comp_err"].size == 0 or rec["comp_err"].max() <= 1.0, (
                rec["k"], rec["comp_err"])
            assert rec["param_err"].max() <= 1.0, (rec["k"], rec["param_err"], rec["gpu_theta"],
                                                   rec["orc_theta"])
