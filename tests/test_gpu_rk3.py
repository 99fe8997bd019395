"""GPU against the FP64 oracle with the three-stage Runge-Kutta update of the
phase field: the step kernel's Euler update is the first stage, two Allen-Cahn
stage launches per step follow.  Bars as for the Euler path (tests/parity.py:
u relative L2 and max |du| / max |u_o| 1e-5 with FP32 populations, 1e-3 with
FP16; p against the oracle's pressure variation; phi 1e-5 / 1e-4; sum phi to
1e-12); batches of such boxes stay bit-identical to the boxes stepped alone.
"""
import numpy as np
import pytest

import oracle as O
from parity import check
from paper_2505_01126_amd import inputs as I

pytestmark = pytest.mark.gpu

TWO_PHASE = dict(rho_l=1.0, rho_g=0.1, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)


@pytest.mark.parametrize("storage,bar_u,bar_phi", [("f32", 1e-5, 1e-5), ("f16", 1e-3, 1e-4)])
def test_runge_kutta_phase_field_matches_oracle(storage, bar_u, bar_phi):
    from paper_2505_01126_amd import lbm

    shape = (24, 17, 70)  # ragged against the 64 x 4 tile and the z-chunk of 5
    phi0, _, _ = I.bubble_pack(shape, 2, 8.0, seed=7)
    u0 = I.solenoidal_field(shape, rms=0.01, k0=2.0, seed=8)
    kw = dict(phi0=phi0, u0=u0, modes=I.forcing_modes(1e-5, seed=9), **TWO_PHASE)
    print(f"case rk3 shape={shape} storage={storage}", flush=True)
    g = lbm.Lattice(shape, 0.6, storage=storage, zchunk=5, ac_rk3=True, **kw)
    r0 = g.reduce()
    g.step(120)
    m = {k: v.double().cpu().numpy() for k, v in g.moments().items()}
    r1 = g.reduce()
    g.close()
    o = O.Oracle(shape, 0.6, ac_rk3=True, **kw)
    o.step(120)
    mo = o.moments()
    err = check(m, mo, storage, "rk3", u_bar=bar_u, phi_bar=bar_phi, drho=0.9)
    dphi = err["phi_max_abs"]
    oe = O.Oracle(shape, 0.6, **kw)
    oe.step(120)
    de = np.abs(oe.moments()["phi"] - mo["phi"]).max()
    print(f"rk3 {storage}: Euler vs Runge-Kutta oracle: phi {de:.3e}")
    assert de > 10 * dphi  # the GPU follows the Runge-Kutta oracle, not the Euler one
    assert abs(r1[0] - r0[0]) / r0[0] < 1e-12


def test_runge_kutta_batch_bit_identical_and_rejects_mixed_integrators():
    from paper_2505_01126_amd import lbm

    shapes = [(16, 20, 70), (32, 32, 32), (20, 36, 20)]
    boxes = []
    for k, shape in enumerate(shapes):
        phi0, _ = I.droplet(shape, 4.0, 4.0, inside=1.0 if k % 2 == 0 else 0.0)
        boxes.append((shape, phi0, I.random_u(shape, 0.01, seed=30 + k)))

    def make(rk3=True):
        return [lbm.Lattice(s, 0.7, phi0=p, u0=u, storage="f16", ac_rk3=rk3, **TWO_PHASE) for s, p, u in boxes]

    alone = make()
    for g in alone:
        g.step(5)
    members = make()
    b = lbm.Batch(members)
    b.step(2)  # one graph replay
    b.set_tiling(32, 8)
    b.step(3)  # replay + single launch
    for i, g in enumerate(members):
        a, c = alone[i].moments(), g.moments()
        for k in a:
            assert bool((a[k] == c[k]).all()), f"box {i}: field {k} differs"
    b.close()
    other = make(rk3=False)[0]
    with pytest.raises(lbm.LbmError):
        lbm.Batch([alone[0], other])
