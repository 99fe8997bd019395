"""Pin of the oracle's global statistics: each of the ten reductions equals
the same statistic computed with numpy from the oracle's own fields
(out[0] sum phi, [1] sum rho, [2] sum p*, [3..5] sum rho u, [6] 1/2 sum rho
|u|^2, [7] max |u|, [8] max overshoot of phi outside [0, 1], [9] non-finite
sites), with p* = p / (rho c_s^2)."""
import numpy as np
import pytest

import oracle as O
from paper_2505_01126_amd import inputs as I


def test_reductions_equal_numpy_statistics_of_the_fields():
    shape = (16, 18, 20)
    phi0, _ = I.droplet(shape, 5.0, 4.0, seed=6)
    phi0 = phi0 * 1.002 - 0.001  # overshoots on both sides
    u0 = I.random_u(shape, 0.02, seed=7)
    o = O.Oracle(shape, 0.7, phi0=phi0, u0=u0, rho_l=1.0, rho_g=0.2, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)
    o.step(5)
    m = o.moments()
    r = o.reduce()
    rho, u, phi = m["rho"], m["u"], m["phi"]
    pstar = m["p"] / (rho / 3.0)
    u2 = (u ** 2).sum(0)
    expect = [phi.sum(), rho.sum(), pstar.sum(), (rho * u[0]).sum(), (rho * u[1]).sum(), (rho * u[2]).sum(),
              0.5 * (rho * u2).sum(), np.sqrt(u2).max(), max((phi - 1.0).max(), (-phi).max(), 0.0), 0.0]
    for k in range(10):
        assert r[k] == pytest.approx(expect[k], rel=1e-12, abs=1e-15), k
    assert r[8] > 0.0


def test_nonfinite_count_is_the_stencil_support_of_a_nan():
    """One NaN in phi0: the forces of Eq. (8) use g and H of the 27-point
    stencil, so the velocity of exactly the 3^3 sites around it is NaN at t = 0
    (and phi at the site itself): out[9] = 27, and the other statistics skip
    those sites and stay finite."""
    shape = (12, 13, 14)
    phi0, _ = I.droplet(shape, 4.0, 4.0, seed=8)
    phi0[3, 4, 5] = np.nan
    o = O.Oracle(shape, 0.8, phi0=phi0, rho_l=1.0, rho_g=0.1, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)
    r = o.reduce()
    assert r[9] == 27
    assert np.all(np.isfinite(r[:9]))
    u = o.moments()["u"]
    bad = ~np.isfinite(u).all(0)
    assert bad.sum() == 27 and bad[2:5, 3:6, 4:7].all()
