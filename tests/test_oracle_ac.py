"""Pins of the oracle's conservative Allen-Cahn update (Sec. 2.1.1, Eq. 3).

- the tanh profile 1/2 (1 + tanh(2 d / delta)) is the steady state up to an
  O((dx/delta)^2) discretisation error (second order: ~4x smaller at 2 delta);
- a profile of the wrong width relaxes to it (the kappa = 4 D / delta balance
  fixes the argument 2 d / delta, not the printed d / delta);
- a uniform velocity translates the profile at that velocity;
- sum phi is conserved to round-off (flux form);
- the update of step n advects with the velocity of step n - 1 (reading R10).
"""
import numpy as np
import pytest

import oracle as O
from paper_2505_01126_amd import inputs as I

D = 0.05


def _run(phi, u, steps, width):
    for _ in range(steps):
        phi = O.ac_update(phi, u, D, width)
    return phi


def test_tanh_profile_is_steady_to_second_order():
    devs = []
    for width, n in ((4.0, 64), (8.0, 128)):
        sh = (4, 4, n)
        phi0 = I.planar_interface(sh, n / 2, width)
        u = np.zeros((3,) + sh)
        steps = int(1000 * (width / 4.0) ** 2)
        devs.append(np.abs(_run(phi0, u, steps, width) - phi0).max())
    assert devs[0] < 0.01
    assert 3.0 < devs[0] / devs[1] < 5.0, devs


def test_wrong_width_relaxes_to_the_2d_over_delta_profile():
    sh = (4, 4, 64)
    width = 4.0
    z, y, x = I.grid(sh)
    d = 16 - np.abs(x - 32) + 0 * y + 0 * z
    wide = 0.5 * (1 + np.tanh(d / width))          # argument d / delta: twice too wide
    target = I.planar_interface(sh, 32.0, width)   # argument 2 d / delta
    u = np.zeros((3,) + sh)
    relaxed = _run(wide, u, 3000, width)
    steady = _run(target, u, 3000, width)
    assert np.abs(wide - target).max() > 0.1
    assert np.abs(relaxed - target).max() < 0.01
    assert np.abs(relaxed - steady).max() < 1e-4


def test_uniform_velocity_translates_profile():
    sh = (4, 4, 64)
    width = 4.0
    u = np.zeros((3,) + sh)
    u[0] = 0.02
    phi0 = I.planar_interface(sh, 32.0, width)
    phi = _run(phi0, u, 500, width)
    shifted = I.planar_interface(sh, 42.0, width)
    assert np.abs(phi - shifted).max() < 0.01
    # the profile moved by 10 cells, not by 9 or 11
    assert np.abs(phi - I.planar_interface(sh, 41.0, width)).max() > 0.05
    assert np.abs(phi - I.planar_interface(sh, 43.0, width)).max() > 0.05
    assert abs(phi.sum() - phi0.sum()) / phi0.sum() < 1e-14


@pytest.mark.parametrize("seed", [0, 1])
def test_sum_phi_conserved_with_random_velocity(seed):
    rng = np.random.default_rng(seed)
    sh = (9, 11, 13)
    phi = rng.uniform(0, 1, sh)
    u = rng.uniform(-0.05, 0.05, (3,) + sh)
    s0 = phi.sum()
    for _ in range(50):
        phi = O.ac_update(phi, u, D, 4.0)
    assert abs(phi.sum() - s0) / s0 < 1e-14


# the Euler update of the phase field with the velocity the same step computes
# instead of the previous step's (no lag)
PLANTED_LAG = {
    "no lag": ("            } else {\n                orc_ac_update(nx, ny, nz, s->phi, s->uprev, p->mobility, p->width, s->phinew);",
               "            } else {\n                orc_ac_update(nx, ny, nz, s->phi, s->unew, p->mobility, p->width, s->phinew);"),
}


def _slab_from_rest(library=None, accel=0.0):
    """A planar slab (phi = 1 for |x - 24| < 8) at rest, equal densities and
    no surface tension, pushed along x by a uniform body acceleration."""
    shape = (8, 8, 48)
    z, y, x = I.grid(shape)
    phi0 = I.tanh_profile(8.0 - np.abs(x - 24.0) + 0.0 * (y + z), 4.0)
    o = O.Oracle(shape, 0.8, phi0=phi0, rho_l=1.0, rho_g=1.0, sigma=0.0, mobility=0.05, width=4.0, p0=0.0,
                 two_phase=True, library=library)
    a = np.zeros((3,) + shape)
    a[0] = accel
    o.set_accel(a)
    return o, x


def _check_velocity_lag(library=None):
    A = 0.01
    pushed, x = _slab_from_rest(library, A)
    still, _ = _slab_from_rest(library, 0.0)
    pushed.step(1)
    still.step(1)
    # step 0 advects phi with the initial velocity (zero), not with the u^0 = A/2
    # that the same step computes: the push has not reached phi yet
    np.testing.assert_array_equal(pushed.moments()["phi"], still.moments()["phi"])
    np.testing.assert_allclose(pushed.get_uprev()[0], A / 2, rtol=1e-12)
    pushed.step(1)
    still.step(1)
    # step 1 advects it with u^0 = A/2: the slab's centroid moves by A/2 (flux
    # form: the first moment changes by u times the sum of the face values)
    p1, p0 = pushed.moments()["phi"], still.moments()["phi"]
    shift = (x * p1).sum() / p1.sum() - (x * p0).sum() / p0.sum()
    assert abs(shift / (A / 2) - 1.0) < 1e-3, shift


def test_allen_cahn_update_uses_the_previous_steps_velocity():
    """Reading R10: the phase field of step n is advected with u^(n-1) (u^(-1)
    = u0).  A slab at rest pushed by a uniform acceleration A from step 0: the
    Guo velocity of step n is A (n + 1/2), so phi is untouched by the push in
    step 0 and moves by A/2 in step 1."""
    _check_velocity_lag()


@pytest.mark.parametrize("name", sorted(PLANTED_LAG))
def test_velocity_lag_pin_catches_planted_mistakes(name, tmp_path):
    from oracle import build as OB

    lib = O.load(OB.build_planted([PLANTED_LAG[name]], str(tmp_path)))
    with pytest.raises(AssertionError):
        _check_velocity_lag(lib)
