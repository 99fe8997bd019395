"""The int32 fixed-point phase field (phi = q 2^-30) against the FP64 oracle.

The oracle keeps phi in FP64; the GPU rounds phi0 to the fixed-point grid and
every face and link flux of the Allen-Cahn update once to that grid (half a
quantum, 4.7e-10, per flux), so it stays within the FP32-storage bars of the
FP64-phi path: u relative L2 and max |du| / max |u_o| below 1e-5 (FP32
populations) or 1e-3 (FP16), p against the oracle's pressure variation, phi
within 1e-5 (FP32) or 1e-3 (FP16).  The integer sum of q is conserved
exactly, so sum phi reported by the reduction equals, bit for bit and at
every step, the sum of the rounded initial field computed on the host in
integer arithmetic.
"""
import numpy as np
import pytest

import oracle as O
from paper_2505_01126_amd import inputs as I
from parity import check

pytestmark = pytest.mark.gpu

TWO_PHASE = dict(rho_l=1.0, rho_g=0.1, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)


def _lattice(shape, tau, storage, phi_storage="fix32", **kw):
    from paper_2505_01126_amd import lbm

    print(f"case shape={shape} tau={tau} storage={storage} phi={phi_storage}", flush=True)
    return lbm.Lattice(shape, tau, storage=storage, phi_storage=phi_storage, **kw)


def _fields(g):
    return {k: v.double().cpu().numpy() for k, v in g.moments().items()}


def _host_sum_fixed(phi0):
    """Sum of phi0 rounded to the 2^-30 grid (round half to even), exact."""
    q = np.rint(np.clip(np.asarray(phi0, dtype=np.float64) * 2.0 ** 30, -2.0 ** 31, 2.0 ** 31 - 1)).astype(np.int64)
    return float(q.sum()) * 2.0 ** -30, q


@pytest.mark.parametrize("storage,bar_u,bar_phi", [("f32", 1e-5, 1e-5), ("f16", 1e-3, 1e-3)])
def test_fixed_point_phi_matches_oracle(storage, bar_u, bar_phi):
    shape = (24, 17, 40)  # ragged against the 64 x 4 tile and the z-chunk of 5
    phi0, _, _ = I.bubble_pack(shape, 2, 8.0, seed=7)
    u0 = I.solenoidal_field(shape, rms=0.01, k0=2.0, seed=8)
    modes = I.forcing_modes(1e-5, seed=9)
    kw = dict(phi0=phi0, u0=u0, modes=modes, **TWO_PHASE)
    g = _lattice(shape, 0.6, storage, zchunk=5, **kw)
    m0 = _fields(g)
    # the initial phi is the fixed-point rounding of phi0, converted back exactly
    _, q = _host_sum_fixed(phi0)
    np.testing.assert_array_equal(m0["phi"], q.astype(np.float64) * 2.0 ** -30)
    g.step(60)
    m = _fields(g)
    g.close()
    o = O.Oracle(shape, 0.6, **kw)
    o.step(60)
    mo = o.moments()
    check(m, mo, storage, "fix32 phi", u_bar=bar_u, phi_bar=bar_phi, drho=0.9)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_fixed_point_phase_volume_exact(storage):
    import bench

    shape, phi0, u0, params, nb = bench.workload(64)
    g = _lattice(shape, 0.515, storage, phi0=phi0, u0=u0, **params)
    expect, _ = _host_sum_fixed(phi0)
    seen = [g.reduce()[0]]
    for n in (1, 10, 89, 200):
        g.step(n)
        r = g.reduce()
        assert r[9] == 0
        seen.append(r[0])
    g.close()
    print(f"fix32 {storage}: sum phi {expect!r}, reduced at 0/1/11/100/300 steps {seen}")
    assert all(v == expect for v in seen)


def test_fixed_point_batch_bit_identical_and_rejects_mixed_phi():
    from paper_2505_01126_amd import lbm

    shapes = [(16, 20, 70), (32, 32, 32), (20, 36, 20)]
    boxes = []
    for k, shape in enumerate(shapes):
        phi0, _ = I.droplet(shape, 4.0, 4.0, inside=1.0 if k % 2 == 0 else 0.0)
        boxes.append((shape, phi0, I.random_u(shape, 0.01, seed=20 + k)))

    def make(phs="fix32"):
        return [_lattice(s, 0.7, "f16", phs, phi0=p, u0=u, **TWO_PHASE) for s, p, u in boxes]

    alone = make()
    for g in alone:
        g.step(5)
    members = make()
    b = lbm.Batch(members)
    b.set_tiling(32, 8)
    b.step(5)
    for i, g in enumerate(members):
        a, c = alone[i].moments(), g.moments()
        for k in a:
            assert bool((a[k] == c[k]).all()), f"box {i}: field {k} differs"
    b.close()
    other = _lattice(shapes[0], 0.7, "f16", "f64", phi0=boxes[0][1], u0=boxes[0][2], **TWO_PHASE)
    with pytest.raises(lbm.LbmError):
        lbm.Batch([alone[0], other])
