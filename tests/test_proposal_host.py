"""Host logic of the proposal trainer (no GPU): the standardisation of the
targets folded into and out of the output layer."""
import numpy as np


def test_standardisation_fold_round_trip():
    """Host logic of the trainer: weights that output t, unfolded to output
    (t - mean) / std and folded back, are the same weights; the unfolded output
    layer maps the last hidden layer to the standardised target."""
    from paper_1606_07872_amd import proposal
    rng = np.random.default_rng(7)
    w = rng.normal(0.0, 0.1, size=329220).astype(np.float32)
    mean = rng.normal(0.0, 2.0, size=4)
    std = rng.uniform(0.2, 5.0, size=4)
    u = proposal.unfold_standardisation(w, mean, std)
    back = proposal.fold_standardisation(u, mean, std)
    np.testing.assert_allclose(back, w, rtol=1e-5, atol=1e-6)
    h2 = rng.uniform(0.0, 1.0, size=256)
    W3, b3 = w[-1028:-4].reshape(4, 256).astype(np.float64), w[-4:].astype(np.float64)
    U3, c3 = u[-1028:-4].reshape(4, 256).astype(np.float64), u[-4:].astype(np.float64)
    np.testing.assert_allclose(U3 @ h2 + c3, (W3 @ h2 + b3 - mean) / std, rtol=1e-5, atol=1e-5)
