"""Pins of the oracle's buoyancy and viscosity-contrast terms.

Buoyancy: the body force (rho - rho_mean) g, with rho_mean the box-mean
density, drives a periodic box without accelerating it as a whole.  At rest
with p* = 0 and no surface tension the first velocity is exactly
(rho - rho_mean) g / (2 rho) up to the second-order viscous correction, and
the box's momentum is zero; with equal densities, or in single phase,
gravity changes nothing; a light bubble rises against g relative to the
liquid.  (Over many steps the velocity-based scheme does not conserve the
box's momentum exactly: the pressure correction and the advection of density
leave a small net force once a hydrostatic pressure has built up.)

Viscosity contrast: tau(phi) = phi tau_l + (1 - phi) tau_g, i.e. the kinematic
viscosity interpolates linearly.  A shear wave in a uniform phase field decays
at exp(-nu(phi) k^2 t) for phi = 0, 1/2, 1; and a layered Kolmogorov flow
(liquid slab in gas, density ratio 10, viscosity ratio 2.5, sinusoidal body
acceleration) relaxes to the steady profile of d/dy (rho nu du/dy) = -rho a(y),
solved here independently on a 16x finer grid.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2505_01126_amd import inputs as I


def test_buoyancy_first_velocity_closed_form():
    shape = (24, 24, 24)
    phi0, _ = I.droplet(shape, 6.0, 4.0, seed=2)  # heavy droplet (phi = 1) in a light gas
    g = (0.0, 0.0, -1e-5)
    o = O.Oracle(shape, 0.8, phi0=phi0, rho_l=1.0, rho_g=0.1, sigma=0.0, mobility=0.05, width=4.0, p0=0.0,
                 gravity=g)
    m = o.moments()
    rho = 0.1 + 0.9 * phi0
    rho_mean = 0.1 + 0.9 * phi0.mean()
    expect = (rho - rho_mean) * g[2] / (2.0 * rho)
    assert max(np.abs(m["u"][0]).max(), np.abs(m["u"][1]).max()) < 1e-12 * np.abs(expect).max()
    err = np.abs(m["u"][2] - expect).max() / np.abs(expect).max()
    assert err < 1e-5  # the viscous correction is second order in g
    assert m["u"][2][12, 12, 12] < 0.0 < m["u"][2][0, 0, 0]  # the droplet falls, the gas rises
    assert abs((rho * m["u"][2]).sum()) < 1e-12 * (rho * np.abs(m["u"][2])).sum()


def test_gravity_inert_without_density_difference():
    shape = (16, 16, 16)
    phi0, _ = I.droplet(shape, 4.0, 4.0, seed=3)
    u0 = I.random_u(shape, 0.01, seed=4)
    base = dict(phi0=phi0, u0=u0, rho_l=1.0, rho_g=1.0, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)
    a = O.Oracle(shape, 0.7, **base)
    b = O.Oracle(shape, 0.7, gravity=(1e-4, -2e-4, 3e-4), **base)
    a.step(20)
    b.step(20)
    np.testing.assert_array_equal(a.moments()["u"], b.moments()["u"])
    c = O.Oracle(shape, 0.7, u0=u0)
    d = O.Oracle(shape, 0.7, u0=u0, gravity=(1e-4, -2e-4, 3e-4))
    c.step(20)
    d.step(20)
    np.testing.assert_array_equal(c.moments()["u"], d.moments()["u"])


def test_light_bubble_rises():
    shape = (32, 24, 24)
    phi0, _ = I.droplet(shape, 5.0, 4.0, seed=5, inside=0.0)
    o = O.Oracle(shape, 0.8, phi0=phi0, rho_l=1.0, rho_g=0.1, sigma=0.01, mobility=0.05, width=4.0, p0=0.0,
                 gravity=(0.0, 0.0, -1e-5))
    z = np.arange(shape[0])[:, None, None] * np.ones(shape)

    def centroid(phi):
        w = np.clip(0.5 - phi, 0.0, None)  # the bubble's core only
        return (w * z).sum() / w.sum()

    z0 = centroid(phi0)
    o.step(1000)
    m = o.moments()
    core = m["phi"] < 0.5
    ub = m["u"][2][core].mean()
    ul = m["u"][2][m["phi"] > 0.99].mean()
    print(f"bubble centroid {z0:.4f} -> {centroid(m['phi']):.4f}, bubble u_z {ub:.3e}, liquid u_z {ul:.3e}")
    assert centroid(m["phi"]) > z0 + 0.1
    assert ub - ul > 1e-5


@pytest.mark.parametrize("phi", [0.0, 0.5, 1.0])
def test_shear_wave_decays_with_phase_viscosity(phi):
    shape = (4, 32, 4)
    tau_l, tau_g, U, steps = 0.8, 0.6, 1e-3, 300
    k = 2.0 * math.pi / shape[1]
    y = np.arange(shape[1])[None, :, None] * np.ones(shape)
    u0 = np.zeros((3,) + shape)
    u0[0] = U * np.sin(k * y)
    o = O.Oracle(shape, tau_l, phi0=np.full(shape, phi), u0=u0, rho_l=1.0, rho_g=0.5, sigma=0.0, mobility=0.05,
                 width=4.0, p0=0.0, tau_g=tau_g)
    o.step(steps)
    ux = o.moments()["u"][0]
    amp = (ux * np.sin(k * y)).sum() / (np.sin(k * y) ** 2).sum()
    nu = (phi * tau_l + (1 - phi) * tau_g - 0.5) / 3.0
    rate = -math.log(amp / U) / steps
    print(f"phi {phi}: decay rate {rate:.6e}, nu k^2 {nu * k * k:.6e}")
    assert rate == pytest.approx(nu * k * k, rel=5e-3)


def _steady_profile(phi_y, rho_l, rho_g, nu_l, nu_g, amp, refine=16):
    """Periodic solution of d/dy (mu du/dy) = -rho a(y), mu = rho nu, rho and nu
    linear in phi, a = amp sin(2 pi y / L), with zero total momentum; phi(y)
    is interpolated (periodic cubic) onto a grid `refine` times finer and the
    second-order conservative difference equation is solved there."""
    L = len(phi_y)
    n = L * refine
    yf = np.arange(n) / refine
    # periodic cubic interpolation of phi through the lattice values
    from scipy.interpolate import CubicSpline

    ys = np.arange(L + 1)
    cs = CubicSpline(ys, np.append(phi_y, phi_y[0]), bc_type="periodic")
    ph = cs(yf)
    rho = rho_g + (rho_l - rho_g) * ph
    mu = rho * (nu_g + (nu_l - nu_g) * np.clip(ph, 0.0, 1.0))
    f = rho * amp * np.sin(2.0 * math.pi * yf / L)
    h = 1.0 / refine
    mh = 0.5 * (mu + np.roll(mu, -1))  # mu at j + 1/2
    A = np.zeros((n, n))
    for j in range(n):
        A[j, j] = -(mh[j] + mh[j - 1]) / h ** 2
        A[j, (j + 1) % n] += mh[j] / h ** 2
        A[j, (j - 1) % n] += mh[j - 1] / h ** 2
    # the operator is singular (constants); replace one row by the momentum condition
    A[0, :] = rho
    rhs = -f.copy()
    rhs[0] = 0.0
    u = np.linalg.solve(A, rhs)
    return u[::refine]


def _layered_flow(library=None):
    """Steady layered Kolmogorov flow of the oracle (liquid slab in gas,
    density ratio 10, tau 1.0 / 0.7, a_x = amp sin(2 pi y / L), 6000 steps)
    against the independent fine-grid solution: (max relative u_x error,
    max |u_y| over max |u_ref|)."""
    shape = (4, 32, 4)
    L = shape[1]
    y = np.arange(L, dtype=np.float64)
    d = L / 4.0 - np.abs(y - L / 2.0)  # slab of half width L/4 centred at L/2
    phi_y = I.tanh_profile(d, 4.0)
    phi0 = np.broadcast_to(phi_y[None, :, None], shape).copy()
    tau_l, tau_g, rho_l, rho_g, amp = 1.0, 0.7, 1.0, 0.1, 2e-6
    modes = np.array([[0, 1, 0, 0.0, -amp, 0, 0, 0, 0]], dtype=np.float64)  # a_x = amp sin(2 pi y / L)
    o = O.Oracle(shape, tau_l, phi0=phi0, rho_l=rho_l, rho_g=rho_g, sigma=0.0, mobility=0.05, width=4.0, p0=0.0,
                 modes=modes, tau_g=tau_g, library=library)
    o.step(6000)
    m = o.moments()
    ux = m["u"][0][0, :, 0]
    phi_end = m["phi"][0, :, 0]
    ref = _steady_profile(phi_end, rho_l, rho_g, (tau_l - 0.5) / 3.0, (tau_g - 0.5) / 3.0, amp)
    err = np.abs(ux - ref).max() / np.abs(ref).max()
    return err, np.abs(m["u"][1]).max() / np.abs(ref).max()


def test_layered_kolmogorov_flow_matches_variable_property_momentum_equation():
    """This also pins the viscous correction F^nu of Eq. (8): without it the
    steady profile moves far outside the bar (next test)."""
    err, uy = _layered_flow()
    print(f"layered flow: rel err {err:.3e}")
    assert uy < 1e-6
    assert err < 2e-2


PLANTED_VISCOUS = {
    "no viscous correction F^nu": ("Fnu *= -(nu / (tau * CS2));", "Fnu *= 0.0;"),
    "F^nu with the wrong sign": ("Fnu *= -(nu / (tau * CS2));", "Fnu *= (nu / (tau * CS2));"),
    "one relaxation time": ("return c * p->tau + (1.0 - c) * p->tau_g;", "return p->tau;"),
}


@pytest.mark.parametrize("name", sorted(PLANTED_VISCOUS))
def test_planted_viscous_mistake_is_caught(name, tmp_path):
    from oracle import build as OB

    lib = O.load(OB.build_planted([PLANTED_VISCOUS[name]], str(tmp_path)))
    err, uy = _layered_flow(lib)
    print(f"{name}: rel err {err:.3e}")
    assert err > 2e-2
