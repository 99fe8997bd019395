"""Pins of the oracle's learned-curvature network (27 -> 64 -> 64 -> 4, tanh).

- fp16 rounding matches IEEE binary16 round-to-nearest-even (numpy float16);
- a network wired as identity blocks reduces to y = tanh(tanh(x)) with fp16
  rounding at the input and after each activation;
- the analytic gradient of the MSE loss matches central differences of the
  forward pass (fp16 emulation off);
- harvested labels on an exact sphere: K = -2/R (phi = 1 inside), n radial
  toward phi = 1, one sample per interface cell.
"""
import numpy as np
import pytest

import oracle as O
from paper_2505_01126_amd import inputs as I

NP = O.MLP_NPARAM


def _split(w):
    W1 = w[:1728].reshape(64, 27)
    b1 = w[1728:1792]
    W2 = w[1792:5888].reshape(64, 64)
    b2 = w[5888:5952]
    W3 = w[5952:6208].reshape(4, 64)
    b3 = w[6208:6212]
    return W1, b1, W2, b2, W3, b3


def test_fp16_rounding_matches_ieee():
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.standard_normal(4000) * np.logspace(-9, 5, 4000),
                        [65504.0, 65519.0, 2.0 ** -24, 3 * 2.0 ** -26, 1e-9, 0.1, -0.333]])
    with np.errstate(over="ignore"):
        ref = v.astype(np.float16).astype(np.float64)
    got = np.array([O.to_half(x) for x in v])
    np.testing.assert_array_equal(got, ref)


def test_identity_wired_network_reduces_to_nested_tanh():
    w = np.zeros(NP)
    W1, b1, W2, b2, W3, b3 = _split(w)
    for j in range(27):
        W1[j, j] = 1.0
    for j in range(64):
        W2[j, j] = 1.0
    W3[0, 0] = 1.0
    W3[1, 5] = 1.0
    W3[2, 26] = -1.0
    b3[3] = 0.25
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, (16, 27))
    y = O.mlp_forward(w, x)
    h = lambda t: np.asarray(t, dtype=np.float64).astype(np.float16).astype(np.float64)
    tt = h(np.tanh(h(np.tanh(h(x)))))
    np.testing.assert_allclose(y[:, 0], tt[:, 0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(y[:, 1], tt[:, 5], rtol=0, atol=1e-15)
    np.testing.assert_allclose(y[:, 2], -tt[:, 26], rtol=0, atol=1e-15)
    np.testing.assert_allclose(y[:, 3], 0.25, rtol=0, atol=0)


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    w = rng.standard_normal(NP) * 0.2
    x = rng.uniform(-1, 1, (8, 27))
    yt = rng.uniform(-1, 1, (8, 4))
    O.mlp_set_fp16(False)
    try:
        loss, g = O.mlp_loss_grad(w, x, yt)
        idx = rng.choice(NP, 60, replace=False)
        idx = np.concatenate([idx, [0, 1727, 1728, 1791, 1792, 5887, 5888, 5951, 5952, 6207, 6208, 6211]])
        eps = 1e-6
        for k in idx:
            wp = w.copy()
            wp[k] += eps
            wm = w.copy()
            wm[k] -= eps
            lp, _ = O.mlp_loss_grad(wp, x, yt)
            lm, _ = O.mlp_loss_grad(wm, x, yt)
            fd = (lp - lm) / (2 * eps)
            assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-9), k
        # the loss itself is the mean squared error of the forward pass
        y = O.mlp_forward(w, x)
        assert loss == pytest.approx(((y - yt) ** 2).sum() / 8, rel=1e-14)
    finally:
        O.mlp_set_fp16(True)


def test_harvest_labels_on_sphere():
    n = 32
    R = 7.0
    phi, c = I.droplet((n, n, n), R, 4.0, center=(16.2, 15.7, 16.4))
    X, Y, cnt = O.harvest(phi, np.array([c]), np.array([R]))
    band = (phi > 0.02) & (phi < 0.98)
    assert cnt == band.sum() == len(X)
    np.testing.assert_allclose(Y[:, 0], -2.0 / R)
    nrm = np.linalg.norm(Y[:, 1:], axis=1)
    np.testing.assert_allclose(nrm, 1.0, atol=1e-14)
    # the centre sample of each stencil is 2 phi - 1 of an interface cell
    assert ((X[:, 13] > -0.96) & (X[:, 13] < 0.96)).all()
    # normals point inward (toward phi = 1): the inner neighbour along n has larger phi
    # bubble labels flip
    Xb, Yb, cb = O.harvest(1 - phi, np.array([c]), np.array([-R]))
    np.testing.assert_allclose(Yb[:, 0], 2.0 / R)
    np.testing.assert_allclose(Yb[:, 1:], -Y[:, 1:], atol=1e-14)


def test_adam_first_steps_closed_form():
    """With a constant gradient g the bias-corrected Adam step is
    lr * g / (|g| + eps) at every step (mhat = g, vhat = g^2)."""
    n = 7
    g = np.array([1e-3, -2.0, 0.5, 3e-5, -7.0, 1.0, 0.0])
    w = np.linspace(-1, 1, n)
    m = np.zeros(n)
    v = np.zeros(n)
    w0 = w.copy()
    lr, eps = 1e-2, 1e-8
    for t in (1, 2, 3):
        w16 = O.adam(w, m, v, g, t, lr=lr, eps=eps)
        step = lr * g / (np.abs(g) + eps)
        np.testing.assert_allclose(w, w0 - t * step, rtol=1e-12, atol=1e-15)
        np.testing.assert_array_equal(w16, w.astype(np.float16).astype(np.float64))
