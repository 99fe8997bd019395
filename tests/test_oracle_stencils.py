"""Pins of the oracle's lattice stencils (Sec. 2.3), curvature and WENO-5.

Stencils: exact on polynomials (gradient up to degree 2, Laplacian and Hessian
up to degree 3), checked against analytic derivatives at interior sites.
WENO-5 (Jiang & Shu 1996): exact on linear data, reduces to the linear
fifth-order upwind combination there, fifth-order convergence on a smooth
monotone function, bounded on a step.  Curvature: on exact tanh spheres the
stencil curvature tends to -2/r as (dx/delta)^2 -> 0 (phi = 1 inside).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2505_01126_amd import inputs as I


def _poly(shape, deg, seed):
    """Random polynomial of total degree `deg` with analytic gradient and Hessian."""
    rng = np.random.default_rng(seed)
    z, y, x = I.grid(shape)
    terms = []
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                terms.append((a, b, c, rng.uniform(-1, 1) * 10.0 ** (-(a + b + c))))
    f = 0.0 * x * y * z
    g = [0.0 * f for _ in range(3)]
    H = [[0.0 * f for _ in range(3)] for _ in range(3)]
    X = [x, y, z]
    for (a, b, c, k) in terms:
        e = [a, b, c]
        f = f + k * x ** a * y ** b * z ** c
        for d in range(3):
            if e[d] == 0:
                continue
            ed = list(e)
            ed[d] -= 1
            g[d] = g[d] + k * e[d] * x ** ed[0] * y ** ed[1] * z ** ed[2]
            for d2 in range(3):
                if ed[d2] == 0:
                    continue
                edd = list(ed)
                edd[d2] -= 1
                H[d][d2] = H[d][d2] + k * e[d] * ed[d2] * x ** edd[0] * y ** edd[1] * z ** edd[2]
    return f, g, H


INTERIOR = (slice(1, -1), slice(1, -1), slice(1, -1))


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_exact_on_quadratics(seed):
    shape = (9, 10, 11)
    f, g, _ = _poly(shape, 2, seed)
    G = O.gradient(f)
    for a in range(3):
        np.testing.assert_allclose(G[a][INTERIOR], g[a][INTERIOR], atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_hessian_and_laplacian_exact_on_cubics(seed):
    shape = (9, 10, 11)
    f, _, H = _poly(shape, 3, seed)
    Hs = O.hessian(f)
    order = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for k, (a, b) in enumerate(order):
        np.testing.assert_allclose(Hs[k][INTERIOR], H[a][b][INTERIOR], atol=1e-11)
    L = O.laplacian(f)
    np.testing.assert_allclose(L[INTERIOR], (H[0][0] + H[1][1] + H[2][2])[INTERIOR], atol=1e-11)


def test_gradient_second_order_on_sine():
    errs = []
    for n in (16, 32):
        z, y, x = I.grid((4, 4, n))
        k = 2 * math.pi / n
        f = np.sin(k * x) + 0 * y + 0 * z
        G = O.gradient(f)
        errs.append(np.abs(G[0] - k * np.cos(k * x)).max() / k)
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.05)


def test_weno5_linear_data_is_exact_and_linear_weights():
    for b in (0.3, -2.0):
        v = [b * k for k in (-2, -1, 0, 1, 2)]
        assert O.weno5(*v) == pytest.approx(0.5 * b, abs=1e-14)
    # with equal smoothness indicators the weights are the linear ones:
    # (2 v-2 - 13 v-1 + 47 v0 + 27 v1 - 3 v2) / 60
    v = [1.0 + 0.7 * k for k in (-2, -1, 0, 1, 2)]
    lin = (2 * v[0] - 13 * v[1] + 47 * v[2] + 27 * v[3] - 3 * v[4]) / 60.0
    assert O.weno5(*v) == pytest.approx(lin, abs=1e-14)


def test_weno5_fifth_order_on_smooth_monotone_data():
    """Flux-difference derivative (h_{i+1/2} - h_{i-1/2}) / dx of point values of
    exp(x) on [0, 1] converges at fifth order (no critical points)."""
    errs = []
    for n in (20, 40, 80):
        dx = 1.0 / n
        xs = np.arange(-4, n + 5) * dx
        v = np.exp(xs)
        err = 0.0
        for i in range(4, n + 4):
            hp = O.weno5(*v[i - 2:i + 3])
            hm = O.weno5(*v[i - 3:i + 2])
            err = max(err, abs((hp - hm) / dx - math.exp(xs[i])))
        errs.append(err)
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(orders) > 4.5, (errs, orders)


def test_weno5_bounded_on_step():
    for v in ([0, 0, 0, 1, 1], [0, 0, 1, 1, 1], [1, 1, 1, 0, 0], [0, 1, 1, 1, 1]):
        h = O.weno5(*map(float, v))
        assert -1e-6 < h < 1 + 1e-6


@pytest.mark.parametrize("R", [6.0, 10.0, 16.0])
def test_fd_curvature_on_exact_sphere(R):
    """On a tanh sphere the stencil curvature equals the level-set curvature
    -2/r up to an O((dx/delta)^2) error: ~2.5 % at delta = 4, ~4x less at delta = 8."""
    n = int(2 * R + 24)
    errs = []
    for width in (4.0, 8.0):
        phi, c = I.droplet((n, n, n), R, width, center=(n / 2 + 0.3, n / 2 - 0.2, n / 2 + 0.1))
        K, nh = O.curvature(phi)
        z, y, x = I.grid(phi.shape)
        r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
        band = (phi > 0.45) & (phi < 0.55)
        errs.append(float((K[band] / (-2.0 / r[band])).mean() - 1.0))
        # normals point toward phi = 1 (inward for a phi = 1 sphere)
        dot = nh[0] * (x - c[0]) + nh[1] * (y - c[1]) + nh[2] * (z - c[2])
        assert (dot[band] < 0).all()
        # a bubble (phi = 0 inside) has the opposite curvature
        K2, _ = O.curvature(1.0 - phi)
        np.testing.assert_allclose(K2[band], -K[band], rtol=1e-12, atol=1e-14)
    assert 0 < errs[0] < 0.03
    assert 2.5 < errs[0] / errs[1] < 4.5
