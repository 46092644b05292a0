"""Pins of the FP64 MLP oracle of the learned proposal against what the
mathematics fixes: finite differences of the loss, closed forms of a linear
network and of the first Adam step, a brute-force patch, and the encoding's
round trip.  CPU only."""
import numpy as np
import pytest

from oracle import mlp

SMALL = (7, 5, 6, 3)


def small_case(seed=0, B=4):
    rng = np.random.default_rng(seed)
    flat = rng.normal(size=mlp.n_params(SMALL))
    X = rng.normal(size=(B, SMALL[0]))
    T = rng.normal(size=(B, SMALL[3]))
    return flat, X, T


def test_param_count_default():
    assert mlp.n_params() == 1024 * 256 + 256 + 256 * 256 + 256 + 4 * 256 + 4 == 329220


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    flat, X, T = small_case(seed)
    _, g = mlp.loss_and_grad(flat, X, T, SMALL)
    h = 1e-6
    for i in range(flat.size):
        e = np.zeros_like(flat)
        e[i] = h
        lp, _ = mlp.loss_and_grad(flat + e, X, T, SMALL)
        lm, _ = mlp.loss_and_grad(flat - e, X, T, SMALL)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_linear_network_closed_form():
    """With every pre-activation positive the network is the affine map
    W3 (W2 (W1 x + b1) + b2) + b3."""
    rng = np.random.default_rng(5)
    W1 = rng.uniform(0.1, 1.0, size=(5, 7))
    W2 = rng.uniform(0.1, 1.0, size=(6, 5))
    W3 = rng.normal(size=(3, 6))
    b1, b2, b3 = rng.uniform(0, 1, 5), rng.uniform(0, 1, 6), rng.normal(size=3)
    flat = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    X = rng.uniform(0.0, 1.0, size=(3, 7))
    y, _ = mlp.forward(flat, X, SMALL)
    want = (W3 @ (W2 @ (W1 @ X.T + b1[:, None]) + b2[:, None]) + b3[:, None]).T
    np.testing.assert_allclose(y, want, rtol=1e-13)
    # at the targets the loss and its gradient vanish
    loss, g = mlp.loss_and_grad(flat, X, y, SMALL)
    assert loss == 0.0 and np.all(g == 0.0)


def test_dead_relu_blocks_gradient():
    flat, X, T = small_case(3)
    W1, b1, *_ = mlp.unpack(flat, SMALL)
    b1[...] = -1e6                       # every first-layer unit off
    _, g = mlp.loss_and_grad(flat, X, T, SMALL)
    gW1, gb1, gW2, gb2, gW3, gb3 = mlp.unpack(g, SMALL)
    # h1 = 0, so nothing upstream of it and nothing multiplying it gets a gradient
    assert np.all(gW1 == 0) and np.all(gb1 == 0) and np.all(gW2 == 0)
    assert np.any(gb3 != 0)


def test_first_adam_step_closed_form():
    """From zero moments the bias-corrected first step is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(7)
    g = rng.normal(size=50)
    w0 = rng.normal(size=50)
    w1, m, v = mlp.adam_step(w0, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    np.testing.assert_allclose(w0 - w1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


@pytest.mark.parametrize("where", ["centre", "top_left", "bottom_right", "right_edge"])
def test_patch_brute_force(where):
    rng = np.random.default_rng(11)
    R = rng.normal(size=(40, 50))
    r, c = {"centre": (20, 25), "top_left": (3, 2), "bottom_right": (39, 49),
            "right_edge": (10, 48)}[where]
    R[r, c] = 3.0
    p = mlp.patch(R, r * 50 + c).reshape(32, 32)
    padded = np.zeros((40 + 64, 50 + 64))
    padded[32:72, 32:82] = R
    want = padded[32 + r - 16:32 + r + 16, 32 + c - 16:32 + c + 16] / 3.0
    np.testing.assert_array_equal(p, want)
    assert p[16, 16] == 1.0


def test_encode_decode_round_trip():
    theta = np.array([0.37, 101.25, 57.5, 4.2])
    t = mlp.encode(theta, 57 * 200 + 100, 200, 0.5, 1.3)
    np.testing.assert_allclose(t, [0.74, np.log(4.2 / 1.3), 1.25, 0.5], rtol=1e-15)
    np.testing.assert_allclose(mlp.decode(t, 57 * 200 + 100, 200, 0.5, 1.3), theta, rtol=1e-15)

