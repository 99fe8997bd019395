"""Pins of the oracle's single-phase lattice-Boltzmann step against closed forms.

- Taylor-Green decay E(t)/E0 = exp(-4 nu k^2 t) with nu = c_s^2 (tau - 1/2)
  (Sec. 2.2), within 0.5 % at 32^3 and second order under diffusive scaling;
- Sum p* and sum j conserved to round-off in a periodic box without force;
- a uniform body force raises u by exactly a per step (Guo forcing, Eq. 5);
- ABC (Sec. 5.1) Beltrami field decays as exp(-nu k^2 t);
- the pressure-based equilibrium is gauge invariant in single phase: a
  constant added to p* leaves u unchanged.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2505_01126_amd import inputs as I


def _tgv_error(n, steps, u0, tau=0.8):
    shape = (4, n, n)
    u, p, k = I.tgv(shape, u0=u0)
    o = O.Oracle(shape, tau, u0=u, pstar0=p, p0=1.0)
    E0 = 0.5 * (o.moments()["u"] ** 2).sum()
    o.step(steps)
    E = 0.5 * (o.moments()["u"] ** 2).sum()
    nu = (tau - 0.5) / 3.0
    exact = math.exp(-4.0 * nu * k * k * steps)
    return E / E0, exact


def test_tgv_decay_32():
    ratio, exact = _tgv_error(32, 200, 0.02)
    assert exact == pytest.approx(0.04576, rel=1e-3)
    assert ratio == pytest.approx(exact, rel=5e-3)


def test_tgv_second_order_diffusive_scaling():
    errs = []
    for n, steps, u0 in ((16, 50, 0.04), (32, 200, 0.02)):
        r, e = _tgv_error(n, steps, u0)
        errs.append(abs(r / e - 1.0))
    assert errs[0] / errs[1] > 3.0, errs


def test_mass_and_momentum_conservation():
    shape = (12, 10, 14)
    u = I.solenoidal_field(shape, rms=0.03, k0=2.0, seed=3)
    o = O.Oracle(shape, 0.6, u0=u, p0=1.0)
    f0 = o.get_f()
    c, _ = O.lattice()
    P0 = f0.sum()
    J0 = np.einsum("ixyz,ia->a", f0, c.astype(float))
    o.step(100)
    f = o.get_f()
    assert abs(f.sum() - P0) / P0 < 1e-13
    J = np.einsum("ixyz,ia->a", f, c.astype(float))
    np.testing.assert_allclose(J, J0, atol=1e-13 * o.N * 0.03)


def test_uniform_force_accelerates_exactly():
    shape = (6, 5, 7)
    a = np.array([1e-5, -2e-5, 0.5e-5])
    modes = np.zeros((1, 9))
    modes[0, 3::2] = a  # k = 0 row: a(x) = Re(A) everywhere
    o = O.Oracle(shape, 0.9, p0=1.0, modes=modes)
    for n in (0, 1, 5):
        if n:
            o.step(n - o.steps)
        u = o.moments()["u"]
        for d in range(3):
            np.testing.assert_allclose(u[d], (n + 0.5) * a[d], rtol=0, atol=1e-15)


def test_abc_beltrami_decay():
    n = 32
    shape = (n, n, n)
    U = 0.005
    u0 = I.abc_field(shape, U)
    tau = 0.8
    o = O.Oracle(shape, tau, u0=u0, p0=1.0)
    steps = 200
    o.step(steps)
    u = o.moments()["u"]
    nu = (tau - 0.5) / 3.0
    k = 2 * math.pi / n
    amp = (u * u0).sum() / (u0 * u0).sum()
    assert amp == pytest.approx(math.exp(-nu * k * k * steps), rel=5e-3)


def test_abc_mode_table_matches_closed_form():
    """The six-row table evaluates to the ABC field: at rest (j = 0) the
    velocity is u = a/2, so u(t = 0) is half the ABC closed form."""
    n = 16
    shape = (n, n, n)
    A = 1e-6
    o = O.Oracle(shape, 1.0, p0=1.0, modes=I.abc_modes(A))
    u = o.moments()["u"]
    np.testing.assert_allclose(u, 0.5 * I.abc_field(shape, A), rtol=0, atol=1e-16)


def test_pressure_gauge_invariance_single_phase():
    shape = (8, 9, 10)
    u = I.solenoidal_field(shape, rms=0.02, k0=2.0, seed=1)
    res = []
    for p0 in (1.0, 2.5):
        o = O.Oracle(shape, 0.7, u0=u, p0=p0, modes=I.forcing_modes(1e-5, seed=2))
        o.step(30)
        res.append(o.moments()["u"])
    np.testing.assert_allclose(res[0], res[1], atol=1e-15)
