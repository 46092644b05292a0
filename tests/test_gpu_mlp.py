"""The learned proposal on the GPU against the FP64 NumPy oracle (oracle/mlp.py):
gradients of the training kernels, one Adam step, batched forward, the
inference kernel of the minor cycle, the recorded training pairs, and lockstep
parity of fits started from the network's proposal."""
import numpy as np
import pytest

import oracle
import skygen
from oracle import mlp as omlp
from parity import PARAM_RTOL, RESID_TOL, param_errors

pytestmark = pytest.mark.gpu

asp = pytest.importorskip("paper_1606_07872_amd")
torch = pytest.importorskip("torch")


def rand_net(seed, scale_out=1.0):
    w = omlp.init_params(np.random.default_rng(seed)).astype(np.float32)
    W1, b1, W2, b2, W3, b3 = omlp.unpack(w)
    W3 *= scale_out
    return w


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def tensor_errors(g, go):
    """Per-tensor max |g - go| / max |go| over the six parameter tensors."""
    out = []
    for a, b in zip(omlp.unpack(g.astype(np.float64)), omlp.unpack(go)):
        out.append(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))
    return np.array(out)


@pytest.mark.parametrize("B", [64, 37])
def test_gradient_matches_oracle(B):
    rng = np.random.default_rng(100 + B)
    w = rand_net(B)
    X = rng.normal(0.0, 0.3, size=(B, 1024)).astype(np.float32)
    T = rng.normal(0.0, 1.0, size=(B, 4)).astype(np.float32)
    net = asp.Mlp(w, max_batch=128)
    loss, g = net.loss_grad(dev(X), dev(T))
    lo, go = omlp.loss_and_grad(w.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    print("B", B, "loss", loss, lo, flush=True)
    assert abs(loss - lo) <= 1e-5 * lo
    err = tensor_errors(g, go)
    print("gradient errors per tensor", err, flush=True)
    assert err.max() <= 1e-4, err
    net.close()


def test_adam_step_matches_oracle():
    rng = np.random.default_rng(7)
    B, lr = 64, 1e-3
    w = rand_net(3)
    X = rng.normal(0.0, 0.3, size=(B, 1024)).astype(np.float32)
    T = rng.normal(0.0, 1.0, size=(B, 4)).astype(np.float32)
    net = asp.Mlp(w, max_batch=B)
    order = dev(np.arange(B), torch.int32)
    net.train(dev(X), dev(T), order, B, lr)
    w1 = net.weights().astype(np.float64)
    _, go = omlp.loss_and_grad(w.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    wo, _, _ = omlp.adam_step(w.astype(np.float64), np.zeros_like(go), np.zeros_like(go), go, 1,
                              lr=lr)
    d = np.abs(w1 - wo)
    # the first step is lr * g / (|g| + eps): well conditioned where |g| >> eps
    big = np.abs(go) > 1e-5
    assert d[big].max() <= 1e-3 * lr + 1e-7, d[big].max()
    assert d.max() <= lr * (1.0 + 1e-3)
    net.close()


def test_forward_matches_oracle_ragged():
    rng = np.random.default_rng(9)
    w = rand_net(4)
    X = rng.normal(0.0, 0.3, size=(300, 1024)).astype(np.float32)
    net = asp.Mlp(w, max_batch=128)
    Y = torch.zeros((300, 4), dtype=torch.float32, device="cuda")
    net.forward(dev(X), Y)
    yo, _ = omlp.forward(w.astype(np.float64), X.astype(np.float64))
    err = np.abs(Y.cpu().numpy() - yo).max() / np.abs(yo).max()
    assert err <= 1e-5, err
    net.close()


def test_bad_sample_index_is_an_error():
    w = rand_net(5)
    net = asp.Mlp(w, max_batch=8)
    X = torch.zeros((10, 1024), dtype=torch.float32, device="cuda")
    T = torch.zeros((10, 4), dtype=torch.float32, device="cuda")
    order = dev(np.array([0, 1, 2, 3, 4, 5, 6, 10]), torch.int32)
    with pytest.raises(asp.AspError):
        net.train(X, T, order, 8)
    net.close()


def test_training_reduces_loss():
    """A learnable task (targets an affine function of the inputs): 300 Adam
    steps must cut the loss at least tenfold."""
    rng = np.random.default_rng(21)
    n = 4096
    X = rng.normal(0.0, 0.3, size=(n, 1024)).astype(np.float32)
    A = rng.normal(0.0, 0.05, size=(1024, 4))
    T = (X @ A + 0.3).astype(np.float32)
    net = asp.Mlp(rand_net(6), max_batch=256)
    order = dev(rng.integers(0, n, size=300 * 128), torch.int32)
    l0, _ = net.loss_grad(dev(X[:256]), dev(T[:256]))
    net.train(dev(X), dev(T), order, 128, 1e-3)
    l1, _ = net.loss_grad(dev(X[:256]), dev(T[:256]))
    print("loss", l0, "->", l1, flush=True)
    assert l1 <= 0.1 * l0
    net.close()


def learned_ctx(f, w, **kw):
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter,
                      max_active=f.max_active, **kw)
    ctx.set_mlp(w)
    ctx.set_init_mode(1)
    return ctx


def test_proposal_kernel_matches_oracle():
    f = skygen.make_c128(1)
    w = rand_net(8, scale_out=0.05)
    ctx = learned_ctx(f, w)
    ab, wb = ctx.psf_gauss()
    for it in range(5):
        R0 = ctx.residual().astype(np.float64)
        rc, idx, val = ctx.find_peak()
        assert rc == 0
        rc, rep = ctx.fit_active_set(idx)
        assert rep["init_source"] == 2
        x = omlp.patch(R0, idx)
        y, _ = omlp.forward(w.astype(np.float64), x[None, :])
        want = omlp.decode(y[0], idx, f.shape[1], R0.flat[idx], wb)
        got = rep["init"]
        print("proposal", got, want, flush=True)
        assert abs(got[0] - want[0]) <= 1e-4 * abs(want[0])
        assert abs(got[1] - want[1]) <= 1e-4 and abs(got[2] - want[2]) <= 1e-4
        assert abs(got[3] - want[3]) <= 1e-4 * want[3]
        ctx.update_residual()
    ctx.close()


def test_lockstep_from_network_start():
    """Fits started from the network's proposal: the oracle, given the same
    proposal and the GPU's pre-step state, must select the same members and
    reach the same parameters and residual."""
    f = skygen.make_c128(2)
    w = rand_net(9, scale_out=0.05)
    ctx = learned_ctx(f, w)
    ab, wb = ctx.psf_gauss()
    orc = oracle.Oracle(f.dirty, gain=f.gain, threshold=f.threshold, max_iter=f.max_iter,
                        max_active=f.max_active, alpha_b=ab, omega_b=wb, cap=f.max_iter + 1)
    peak = float(np.abs(f.dirty).max())
    n_strict = 0
    for it in range(30):
        R0 = ctx.residual()
        comps0 = ctx.components_raw()
        k0, _ = ctx.counts()
        rc, idx, val = ctx.find_peak()
        if rc != 0:
            break
        rc, rep = ctx.fit_active_set(idx)
        ctx.update_residual()
        orc.load_state(R0, comps0, k0)
        orep = orc.step(init=rep["init"])
        assert orep["idx"] == idx
        assert orep["members"] == rep["members"], (it, orep["members"], rep["members"])
        assert orep["start_from_proposal"] == rep["start_from_proposal"], it
        assert orep["used_fallback"] == rep["used_fallback"] or not (orep["converged"] and rep["converged"])
        R1 = ctx.residual().astype(np.float64)
        assert np.abs(R1 - orc.R).max() <= RESID_TOL * peak
        if rep["converged"] and orep["converged"]:
            err = param_errors(rep["theta"], orep["theta"])
            assert err.max() <= 1.0, (it, err)
            n_strict += 1
    assert n_strict >= 20
    ctx.close()


def test_recorded_pairs_match_oracle():
    f = skygen.make_c128(3)
    ctx = asp.Context(f.dirty, f.psf, f.gain, f.threshold, max_iter=f.max_iter,
                      max_active=f.max_active)
    cap = 6
    P = torch.zeros((cap, 1024), dtype=torch.float32, device="cuda")
    T = torch.zeros((cap, 4), dtype=torch.float32, device="cuda")
    F = torch.zeros((cap,), dtype=torch.int32, device="cuda")
    ctx.record(P, T, F)
    ab, wb = ctx.psf_gauss()
    reps, Rs = [], []
    for it in range(8):
        Rs.append(ctx.residual().astype(np.float64))
        rc, idx, val = ctx.find_peak()
        rc, rep = ctx.fit_active_set(idx)
        ctx.update_residual()
        reps.append(rep)
    assert ctx.record_count() == cap
    P, T, F = P.cpu().numpy(), T.cpu().numpy(), F.cpu().numpy()
    for n in range(cap):
        rep, R0 = reps[n], Rs[n]
        want_p = omlp.patch(R0, rep["idx"])
        assert np.abs(P[n] - want_p).max() <= 1e-6 * np.abs(want_p).max()
        want_t = omlp.encode(rep["theta"][0], rep["idx"], f.shape[1], R0.flat[rep["idx"]], wb)
        np.testing.assert_allclose(T[n], want_t, rtol=1e-6, atol=1e-6)
        assert F[n] == (int(rep["converged"]) | (int(rep["used_fallback"]) << 1))
    ctx.record(None, None, None)
    ctx.close()


def test_trained_network_cuts_lm_trials():
    """What the trained network gains over the simple values.  Training pairs
    are recorded on the device from plain runs of six 1024 x 1024 fields and
    the network is trained by the library's kernels; then, on a held-out field
    run in learned mode, every pre-step state is fitted by the oracle twice --
    from the simple values and from the device's proposal -- so both fits see
    the identical problem.  The learned start must need clearly fewer LM trials
    and, where the fit is not degenerate, reach the same component."""
    from paper_1606_07872_amd import proposal
    fields = [skygen.make_c1024(1001 + i) for i in range(6)]
    X, T = proposal.record_fields(fields, 1500, torch)
    print("training pairs", X.shape[0], flush=True)
    w, losses, val = proposal.train(X, T, 20, 256, 1e-3, 1, torch)
    print("losses", losses[0], losses[-1], "validation", val, flush=True)
    assert losses[-1] < 0.6 * losses[0]
    f = skygen.make_c1024(1000)
    ctx = learned_ctx(f, w)
    ab, wb = ctx.psf_gauss()
    orc = oracle.Oracle(f.dirty, gain=f.gain, threshold=f.threshold, max_iter=f.max_iter,
                        max_active=f.max_active, alpha_b=ab, omega_b=wb, cap=f.max_iter + 1)
    tr_plain, tr_learned, same = [], [], 0
    for it in range(30):
        R0 = ctx.residual()
        comps0 = ctx.components_raw()
        k0, _ = ctx.counts()
        rc, idx, val = ctx.find_peak()
        rc, rep = ctx.fit_active_set(idx)
        ctx.update_residual()
        orc.load_state(R0, comps0, k0)
        p = orc.step()
        orc.load_state(R0, comps0, k0)
        q = orc.step(init=rep["init"])
        tr_plain.append(p["lm_iters"])
        tr_learned.append(q["lm_iters"])
        same += bool(np.all(param_errors(p["theta"][:1], q["theta"][:1]) <= 1.0))
    print("mean trials plain", np.mean(tr_plain), "learned", np.mean(tr_learned), "same", same,
          flush=True)
    assert np.mean(tr_learned) <= 0.8 * np.mean(tr_plain)
    assert same >= 15
    ctx.close()
