"""Pins of the oracle's single-site pieces against closed-form lattice identities.

D3Q27 moment identities, the pressure-based equilibrium moments (Sec. 2.2),
the Guo forcing moments (Eq. 5) and the regularised collision (Eqs. 6-7):
each check uses a closed form that is not the formula the oracle evaluates.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

CS2 = 1.0 / 3.0


def test_lattice_weights_exact_moments():
    c, w = O.lattice()
    # weights are 8/27, 2/27, 1/54, 1/216 by speed class
    fr = {0: Fraction(8, 27), 1: Fraction(2, 27), 2: Fraction(1, 54), 3: Fraction(1, 216)}
    for i in range(27):
        n2 = int((c[i] ** 2).sum())
        assert w[i] == float(fr[n2])
    W = [fr[int((c[i] ** 2).sum())] for i in range(27)]
    assert sum(W) == 1
    for a in range(3):
        assert sum(W[i] * int(c[i, a]) for i in range(27)) == 0
        for b in range(3):
            m2 = sum(W[i] * int(c[i, a]) * int(c[i, b]) for i in range(27))
            assert m2 == (Fraction(1, 3) if a == b else 0)
    # fourth-order isotropy: sum w c_x^4 = 3 c_s^4, sum w c_x^2 c_y^2 = c_s^4
    assert sum(W[i] * int(c[i, 0]) ** 4 for i in range(27)) == Fraction(1, 3)
    assert sum(W[i] * int(c[i, 0]) ** 2 * int(c[i, 1]) ** 2 for i in range(27)) == Fraction(1, 9)
    # opposite directions pair up as i <-> 26 - i, rest at 13
    assert (c[13] == 0).all()
    for i in range(27):
        assert (c[26 - i] == -c[i]).all()


def _moments(f, c):
    m0 = f.sum()
    m1 = (f[:, None] * c).sum(axis=0)
    m2 = np.einsum("i,ia,ib->ab", f, c, c)
    return m0, m1, m2


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    c, _ = O.lattice()
    c = c.astype(float)
    p = rng.uniform(-0.5, 2.0)
    u = rng.uniform(-0.1, 0.1, 3)
    m0, m1, m2 = _moments(O.feq(p, u), c)
    assert m0 == pytest.approx(p, abs=1e-15)
    np.testing.assert_allclose(m1, u, atol=1e-16)
    np.testing.assert_allclose(m2, p * CS2 * np.eye(3) + np.outer(u, u), atol=1e-16)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_guo_moments(seed):
    rng = np.random.default_rng(seed)
    c, _ = O.lattice()
    c = c.astype(float)
    u = rng.uniform(-0.1, 0.1, 3)
    a = rng.uniform(-1e-3, 1e-3, 3)
    m0, m1, m2 = _moments(O.guo(u, a), c)
    assert abs(m0) < 1e-18
    np.testing.assert_allclose(m1, a, atol=1e-18)
    np.testing.assert_allclose(m2, np.outer(u, a) + np.outer(a, u), atol=1e-18)


def _random_f(rng, c):
    p = rng.uniform(0.8, 1.2)
    u = rng.uniform(-0.05, 0.05, 3)
    f = O.feq(p, u) * (1.0 + rng.uniform(-0.05, 0.05, 27))
    return f


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_collision_invariants_and_closed_form_a2(seed):
    rng = np.random.default_rng(seed)
    c, _ = O.lattice()
    c = c.astype(float)
    f = _random_f(rng, c)
    a = rng.uniform(-1e-3, 1e-3, 3)
    p, j, Pi = _moments(f, c)
    u = j + 0.5 * a
    tau = rng.uniform(0.51, 2.0)
    fp, a2 = O.collide(f, u, a, tau)
    # mass-like invariant and momentum change by the force
    q0, q1, q2 = _moments(fp, c)
    assert q0 == pytest.approx(p, abs=1e-14)
    np.testing.assert_allclose(q1, j + a, atol=1e-15)
    # a^(2) in closed form: Pi - c_s^2 p I - u u + (u a + a u)/2
    A = Pi - CS2 * p * np.eye(3) - np.outer(u, u) + 0.5 * (np.outer(u, a) + np.outer(a, u))
    sym = np.array([A[0, 0], A[1, 1], A[2, 2], A[0, 1], A[0, 2], A[1, 2]])
    np.testing.assert_allclose(a2, sym, atol=1e-15)
    # the post-collision stress relaxes the non-equilibrium part by (1 - 1/tau)
    expect = CS2 * p * np.eye(3) + np.outer(u, u) + (1 - 1 / tau) * A + 0.5 * (np.outer(u, a) + np.outer(a, u))
    np.testing.assert_allclose(q2, expect, atol=1e-14)


def test_collision_tau_one_is_equilibrium_plus_half_force():
    rng = np.random.default_rng(7)
    c, _ = O.lattice()
    f = _random_f(rng, c.astype(float))
    a = np.array([1e-4, -2e-4, 3e-4])
    j = (f[:, None] * c).sum(axis=0)
    u = j + 0.5 * a
    fp, _ = O.collide(f, u, a, 1.0)
    np.testing.assert_allclose(fp, O.feq(f.sum(), u) + 0.5 * O.guo(u, a), atol=1e-16)


def test_regularisation_keeps_equilibrium_fixed():
    u = np.array([0.03, -0.01, 0.02])
    f = O.feq(1.1, u)
    fp, a2 = O.collide(f, u, np.zeros(3), 0.7)
    np.testing.assert_allclose(a2, 0.0, atol=1e-16)
    np.testing.assert_allclose(fp, f, atol=1e-16)


def test_regularisation_filters_ghost_moments():
    """A perturbation orthogonal to the Hermite basis up to second order (a
    third-order 'ghost' mode) is removed entirely by the regularised collision."""
    c, w = O.lattice()
    c = c.astype(float)
    u = np.zeros(3)
    # ghost: w_i c_x^2 c_y^2 c_z^2 made orthogonal (plain sum over i) to the
    # polynomials 1, c_a, c_a c_b - c_s^2 delta_ab, so it carries no p*, j or a^(2)
    g = w * (c[:, 0] ** 2 * c[:, 1] ** 2 * c[:, 2] ** 2)
    basis = [np.ones(27)] + [c[:, a] for a in range(3)] + [
        (c[:, a] * c[:, b] - (CS2 if a == b else 0.0)) for a in range(3) for b in range(a, 3)]
    B = np.array(basis).T
    coef, *_ = np.linalg.lstsq(B, g, rcond=None)
    ghost = g - B @ coef
    assert np.abs(ghost).max() > 1e-3
    f = O.feq(1.0, u) + 1e-3 * ghost
    fp, _ = O.collide(f, u, np.zeros(3), 0.8)
    # the ghost is not in the span, so the regularised result is the plain equilibrium
    np.testing.assert_allclose(fp, O.feq(f.sum(), u), atol=1e-15)
