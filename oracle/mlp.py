"""FP64 NumPy oracle of the learned start-value proposal -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark may import this
module.  It shares no code with the HIP library.

The proposal replaces the simple initial values of Sect. 3 (the residual peak
and the main-lobe width) for the new component of a fit.  A multilayer
perceptron maps the residual patch around the peak to a start point; the LM fit
of Sect. 3 then runs from it and decides whether the proposal is kept: if that
fit does not converge, or ends with a new component of amplitude zero, the
simple values are fitted instead (that rule lives in the C oracle's step).

Network (sizes ``dims = (d0, d1, d2, d3)``, by default (1024, 256, 256, 4)):
    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3,
with the parameters flattened in the order W1 (d1 x d0, row-major), b1, W2
(d2 x d1), b2, W3 (d3 x d2), b3.  The loss of a batch is the mean over samples
and outputs of (y - t)^2.

Patch and targets (the encoding of a fit in the network's terms):
    x = the 32 x 32 residual patch, rows r*-16 .. r*+15 and columns c*-16 ..
        c*+15 around the peak pixel (r*, c*), zero outside the image, divided
        by the residual at the peak;
    t = (a / R[p*], log(s / omega_b), x_fit - c*, y_fit - r*)
for the new component's fitted (a, x, y, s) in convolved space.
"""
from __future__ import annotations

import numpy as np

DIMS = (1024, 256, 256, 4)
PATCH = 32
HALF = 16


def n_params(dims=DIMS) -> int:
    d0, d1, d2, d3 = dims
    return d1 * d0 + d1 + d2 * d1 + d2 + d3 * d2 + d3


def unpack(flat, dims=DIMS):
    """Views (W1, b1, W2, b2, W3, b3) into the flat parameter vector."""
    d0, d1, d2, d3 = dims
    flat = np.asarray(flat)
    out, o = [], 0
    for shape in ((d1, d0), (d1,), (d2, d1), (d2,), (d3, d2), (d3,)):
        n = int(np.prod(shape))
        out.append(flat[o:o + n].reshape(shape))
        o += n
    assert o == flat.size, (o, flat.size)
    return out


def forward(flat, X, dims=DIMS):
    """Outputs (B, d3) and the activations needed by the backward pass."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(flat, dtype=np.float64), dims)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3.T + b3
    return y, (X, z1, h1, z2, h2)


def loss_and_grad(flat, X, T, dims=DIMS):
    """Mean squared error of a batch and its gradient, by the chain rule written
    out layer by layer (reverse order of ``forward``)."""
    flat = np.asarray(flat, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(flat, dims)
    y, (X, z1, h1, z2, h2) = forward(flat, X, dims)
    T = np.asarray(T, dtype=np.float64)
    B, d3 = y.shape
    diff = y - T
    loss = float(np.sum(diff * diff) / (B * d3))
    dy = 2.0 * diff / (B * d3)
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dh2 = dy @ W3
    dz2 = dh2 * (z2 > 0.0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0.0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    grad = np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return loss, grad


def adam_step(flat, m, v, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) at step t >= 1; returns new (flat, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(rng, dims=DIMS) -> np.ndarray:
    """He-uniform weights and zero biases, drawn from ``rng`` (FP32-representable)."""
    parts = []
    d = list(dims)
    for i in range(3):
        fan_in, fan_out = d[i], d[i + 1]
        lim = np.sqrt(6.0 / fan_in) if i < 2 else np.sqrt(3.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=(fan_out, fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def patch(R, idx: int) -> np.ndarray:
    """The 32 x 32 patch around pixel idx of the row-major image R, zero outside
    the image, divided by R at idx (1024 values, row-major)."""
    H, W = R.shape
    r0, c0 = divmod(int(idx), W)
    peak = float(R[r0, c0])
    out = np.zeros((PATCH, PATCH), dtype=np.float64)
    for i in range(PATCH):
        r = r0 - HALF + i
        if r < 0 or r >= H:
            continue
        for j in range(PATCH):
            c = c0 - HALF + j
            if 0 <= c < W:
                out[i, j] = float(R[r, c]) / peak
    return out.ravel()


def encode(theta, idx: int, W: int, peak: float, omega_b: float) -> np.ndarray:
    """Targets of a fitted (a, x, y, s) for a peak at idx with residual `peak`."""
    a, x, y, s = (float(v) for v in theta)
    r0, c0 = divmod(int(idx), W)
    return np.array([a / peak, np.log(s / omega_b), x - c0, y - r0])


def decode(out, idx: int, W: int, peak: float, omega_b: float) -> np.ndarray:
    """The proposal (a, x, y, s) a network output stands for (inverse of encode)."""
    r0, c0 = divmod(int(idx), W)
    o = [float(v) for v in out]
    return np.array([o[0] * peak, c0 + o[2], r0 + o[3], omega_b * np.exp(o[1])])
