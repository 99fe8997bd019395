"""Pins of the oracle's three-stage Runge-Kutta option for the Allen-Cahn update.

With equal densities and no surface tension the lattice flow stays uniform,
so the phase field is advected by a constant velocity and the right-hand side
L(phi) of Eq. (3) is a fixed function of phi.  Scaling the velocity and the
mobility by s and the step count by 1/s is then the same discretisation in
space with a time step of s: the difference from a run at s = 1/64 falls by 8
per halving of s with the Runge-Kutta stages (third order) and by 2 with the
Euler step (first order).  A WENO-advected interface with no diffusion keeps
its overshoots an order of magnitude smaller than with the Euler step, and
both conserve sum phi to round-off.
"""
import numpy as np
import pytest

import oracle as O
from paper_2505_01126_amd import inputs as I

SHAPE = (4, 4, 32)


def _advect(phi0, s, rk3, T=40, U=0.4, D=0.0):
    u0 = np.zeros((3,) + SHAPE)
    u0[0] = U * s
    o = O.Oracle(SHAPE, 0.8, phi0=phi0, u0=u0, rho_l=1.0, rho_g=1.0, sigma=0.0, mobility=D * s, width=4.0, p0=1.0,
                 ac_rk3=rk3)
    r0 = o.reduce()
    o.step(int(round(T / s)))
    return o.moments()["phi"], r0, o.reduce()


@pytest.mark.parametrize("rk3,order", [(True, 3), (False, 1)])
def test_time_order_of_the_allen_cahn_integrator(rk3, order):
    x = np.arange(SHAPE[2])[None, None, :] * np.ones(SHAPE)
    phi0 = 0.5 + 0.2 * np.sin(2.0 * np.pi * x / SHAPE[2])
    ref = _advect(phi0, 1.0 / 64.0, rk3)[0]
    errs = [np.abs(_advect(phi0, s, rk3)[0] - ref).max() for s in (0.5, 0.25, 0.125)]
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    print(f"rk3={rk3}: errors {errs}, ratios {ratios}")
    for r in ratios:
        assert r == pytest.approx(2.0 ** order, rel=0.1)


def test_runge_kutta_keeps_advected_interface_bounded():
    phi0 = I.planar_interface(SHAPE, 16.0, 4.0, axis=2)
    over = {}
    for rk3 in (False, True):
        phi, r0, r1 = _advect(phi0, 1.0, rk3, T=300, U=0.3)
        over[rk3] = max(-phi.min(), phi.max() - 1.0)
        assert abs(r1[0] - r0[0]) / r0[0] < 1e-13
    print(f"overshoot after 300 steps: Euler {over[False]:.3e}, Runge-Kutta {over[True]:.3e}")
    assert over[True] < 0.1 * over[False]
    assert over[True] < 2e-3
