"""GPU against the FP64 oracle with buoyancy, a viscosity contrast and a
density ratio of 100 (the two-phase benchmark ratio of Sec. 4).

Buoyancy is the body force (rho - rho_mean) g with rho_mean the box-mean
density; the viscosity contrast is tau(phi) = phi tau_l + (1 - phi) tau_g.
Bars as for the other two-phase parity tests (tests/parity.py): u relative L2
and max |du| / max |u_o| below 1e-5 with FP32 populations (1e-3 with FP16),
p against the oracle's pressure variation, phi within 1e-5 (1e-4 with FP16).
"""
import numpy as np
import pytest

import oracle as O
from paper_2505_01126_amd import inputs as I
from parity import check

pytestmark = pytest.mark.gpu


def _run(shape, tau, steps, storage="f32", zchunk=0, **kw):
    from paper_2505_01126_amd import lbm

    print(f"case shape={shape} tau={tau} steps={steps} storage={storage} "
          f"gravity={kw.get('gravity')} tau_g={kw.get('tau_g')} ratio={kw['rho_l'] / kw['rho_g']:g}", flush=True)
    g = lbm.Lattice(shape, tau, storage=storage, zchunk=zchunk, **kw)
    g.step(steps)
    m = {k: v.double().cpu().numpy() for k, v in g.moments().items()}
    r = g.reduce()
    g.close()
    o = O.Oracle(shape, tau, **kw)
    o.step(steps)
    return m, r, o.moments(), o.reduce()


def _two_bubbles(shape):
    nz, ny, nx = shape
    a, _ = I.droplet(shape, 5.0, 4.0, center=(nx * 0.3, ny * 0.5, nz * 0.35), inside=0.0)
    b, _ = I.droplet(shape, 4.0, 4.0, center=(nx * 0.75, ny * 0.4, nz * 0.7), inside=0.0)
    return np.minimum(a, b)


@pytest.mark.parametrize("gravity,tau_g,storage,bar_u,bar_phi", [
    ((0.0, 0.0, -1e-5), 0.0, "f32", 1e-5, 1e-5),
    ((0.0, 0.0, 0.0), 0.6, "f32", 1e-5, 1e-5),
    ((2e-6, -3e-6, -1e-5), 0.6, "f32", 1e-5, 1e-5),
    ((2e-6, -3e-6, -1e-5), 0.6, "f16", 1e-3, 1e-4),
])
def test_buoyancy_and_viscosity_contrast_match_oracle(gravity, tau_g, storage, bar_u, bar_phi):
    shape = (26, 20, 70)  # ragged against the 64 x 4 tile and the z-chunk of 8
    phi0 = _two_bubbles(shape)
    u0 = I.random_u(shape, 0.005, seed=11)
    kw = dict(phi0=phi0, u0=u0, rho_l=1.0, rho_g=0.1, sigma=0.01, mobility=0.05, width=4.0, p0=0.0,
              gravity=gravity, tau_g=tau_g)
    m, r, mo, ro = _run(shape, 0.8, 150, storage, zchunk=8, **kw)
    check(m, mo, storage, f"g {gravity} tau_g {tau_g}", u_bar=bar_u, phi_bar=bar_phi, drho=0.9)
    assert abs(r[0] - ro[0]) / ro[0] < 1e-12
    assert r[9] == 0


@pytest.mark.parametrize("storage,bar_u", [("f32", 1e-5), ("f16", 1e-3)])
def test_density_ratio_100_matches_oracle(storage, bar_u):
    shape = (32, 32, 32)
    phi0, _ = I.droplet(shape, 8.0, 4.0, seed=4)  # heavy droplet, ratio 100 (Sec. 4 benchmark)
    u0 = I.random_u(shape, 0.002, seed=12)
    kw = dict(phi0=phi0, u0=u0, rho_l=1.0, rho_g=0.01, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)
    m, r, mo, ro = _run(shape, 0.8, 300, storage, **kw)
    print(f"ratio 100 {storage}: max |u| {np.abs(mo['u']).max():.2e}")
    check(m, mo, storage, "ratio 100", u_bar=bar_u, phi_bar=1e-5 if storage == "f32" else 1e-3, drho=0.99)
    assert r[9] == 0


def test_layered_kolmogorov_flow_matches_oracle():
    shape = (8, 32, 8)  # the library needs 8 sites per axis
    L = shape[1]
    y = np.arange(L, dtype=np.float64)
    phi_y = I.tanh_profile(L / 4.0 - np.abs(y - L / 2.0), 4.0)
    phi0 = np.broadcast_to(phi_y[None, :, None], shape).copy()
    amp = 2e-6
    modes = np.array([[0, 1, 0, 0.0, -amp, 0, 0, 0, 0]], dtype=np.float64)
    kw = dict(phi0=phi0, rho_l=1.0, rho_g=0.1, sigma=0.0, mobility=0.05, width=4.0, p0=0.0, modes=modes, tau_g=0.7)
    m, r, mo, ro = _run(shape, 1.0, 1000, "f32", **kw)
    check(m, mo, "f32", "layered flow after 1000 steps", phi_bar=1e-5, drho=0.9)
