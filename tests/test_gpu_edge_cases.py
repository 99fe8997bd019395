"""Edge cases of the step against the FP64 oracle: the smallest box, every
z-chunk length down to one plane, zero steps, and the largest boxes the ABI
accepts.

* 8^3 (the smallest box): the phase-field stencils (WENO-5 radius 3) reach
  across most of the box and wrap; z-chunks of 1, 3 (ragged: 3 + 3 + 2) and 8
  planes, element by element against the oracle and bit-identical to each
  other.
* zero steps leave every field bit for bit and the step count unchanged;
  negative step counts are rejected.
* equal densities and no surface tension (the degenerate two-phase case): the
  coupled kernel's flow is the single-phase kernel's.
* nx * ny = 2^24 (the largest xy plane, FP32: the largest per-plane buffer
  range of the population loads) and nx * ny * nz = 2^30 (the largest box,
  FP16: 148 GiB of state, population offsets beyond 2^32 elements) after two
  steps, on sampled sites: the oracle recomputes each site exactly on a 24^3
  periodic window of the initial fields (one site's state after two steps
  depends only on the initial fields within a few cells; with nz = 8 the
  window holds three periods of the box and is exact for the same reason).
  The largest box also checks sum phi at t = 0 against numpy and its
  conservation, and that no site turned non-finite.
Bars as elsewhere (tests/parity.py): u relative L2 and max |du| / max |u_o|
below 1e-5 with FP32 populations and 1e-3 with FP16, p against the oracle's
pressure variation, phi within 1e-5 (FP32) / 1e-4 (FP16).
"""
import gc

import numpy as np
import pytest

import oracle as O
from paper_2505_01126_amd import inputs as I
from parity import check

pytestmark = pytest.mark.gpu

TWO_PHASE = dict(rho_l=1.0, rho_g=0.1, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)
W = 24


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_smallest_box_every_zchunk():
    from paper_2505_01126_amd import lbm

    shape = (8, 8, 8)
    phi0, _ = I.droplet(shape, 2.5, 4.0, center=(3.7, 4.2, 4.6))
    u0 = I.random_u(shape, 0.01, seed=61)
    modes = I.forcing_modes(1e-5, seed=62)
    kw = dict(phi0=phi0, u0=u0, modes=modes, **TWO_PHASE)
    o = O.Oracle(shape, 0.7, **kw)
    o.step(12)
    mo, ro = o.moments(), o.reduce()
    first = None
    for zchunk in (1, 3, 8):
        print(f"case smallest box shape={shape} zchunk={zchunk}", flush=True)
        g = lbm.Lattice(shape, 0.7, zchunk=zchunk, **kw)
        g.step(12)
        m = {k: v.double().cpu().numpy() for k, v in g.moments().items()}
        r = g.reduce()
        g.close()
        check(m, mo, "f32", f"8^3 zchunk {zchunk}", phi_bar=1e-5, drho=0.9)
        assert abs(r[0] - ro[0]) < 1e-10 * abs(ro[0])
        # the z-chunk only splits the work: every site does the same arithmetic
        if first is None:
            first = m
        for k in m:
            assert np.array_equal(m[k], first[k]), f"zchunk {zchunk}: field {k} differs from zchunk 1"


def test_smallest_box_single_phase_half_storage():
    from paper_2505_01126_amd import lbm

    shape = (8, 8, 8)
    u0 = I.random_u(shape, 0.02, seed=63)
    modes = I.forcing_modes(1e-4, seed=64)
    print(f"case smallest box single phase f16 shape={shape} zchunk=1", flush=True)
    g = lbm.Lattice(shape, 0.6, u0=u0, modes=modes, storage="f16", zchunk=1, p0=1.0)
    g.step(20)
    m = {k: v.double().cpu().numpy() for k, v in g.moments().items()}
    g.close()
    o = O.Oracle(shape, 0.6, u0=u0, modes=modes, p0=1.0)
    o.step(20)
    check(m, o.moments(), "f16", "8^3 single phase")


def test_zero_steps_change_nothing():
    from paper_2505_01126_amd import lbm

    shape = (10, 12, 70)
    phi0, _ = I.droplet(shape, 4.0, 4.0, seed=65)
    print(f"case zero steps shape={shape}", flush=True)
    g = lbm.Lattice(shape, 0.7, phi0=phi0, u0=I.random_u(shape, 0.01, seed=66), storage="f16", **TWO_PHASE)
    g.step(3)
    a = {k: v.clone() for k, v in g.moments().items()}
    g.step(0)
    assert g.steps == 3
    b = g.moments()
    for k in a:
        assert bool((a[k] == b[k]).all()), f"field {k} changed"
    with pytest.raises(lbm.LbmError):
        g.step(-1)
    assert g.steps == 3
    g.close()


def test_equal_densities_without_tension_match_single_phase():
    """With equal densities and no surface tension the coupled step carries no
    phase-field force: its flow matches the single-phase kernel's (FP32
    round-off of the density mix rho(phi) aside) and the oracle's."""
    from paper_2505_01126_amd import lbm

    shape = (12, 14, 70)
    phi0, _ = I.droplet(shape, 4.0, 4.0, seed=3)
    u0 = I.random_u(shape, 0.02, seed=4)
    modes = I.forcing_modes(1e-4, seed=5)
    print(f"case equal densities, sigma 0 vs single phase shape={shape}", flush=True)
    a = lbm.Lattice(shape, 0.7, phi0=phi0, u0=u0, modes=modes, rho_l=1.0, rho_g=1.0, sigma=0.0, mobility=0.05,
                    width=4.0, p0=0.0, zchunk=8)
    b = lbm.Lattice(shape, 0.7, u0=u0, modes=modes, rho_l=1.0, p0=0.0, zchunk=8)
    a.step(30)
    b.step(30)
    ma = {k: v.double().cpu().numpy() for k, v in a.moments().items()}
    mb = {k: v.double().cpu().numpy() for k, v in b.moments().items()}
    a.close()
    b.close()
    o = O.Oracle(shape, 0.7, u0=u0, modes=modes, rho_l=1.0, p0=0.0)
    o.step(30)
    mo = o.moments()
    del ma["phi"], mo["phi"], mb["phi"]
    check(ma, mb, "f32", "equal densities: two-phase vs single-phase kernel")
    check(ma, mo, "f32", "equal densities: two-phase kernel vs oracle")


def _window(a, origin, shape):
    idx = [np.arange(o, o + W) % n for o, n in zip(origin, shape)]
    return a[np.ix_(*idx)]


def _sampled_parity(shape, storage, tau, phi0, u0, modes, pts, extra_check=None):
    import torch

    from paper_2505_01126_amd import lbm

    print(f"case largest box shape={shape} storage={storage}: stepping", flush=True)
    g = lbm.Lattice(shape, tau, phi0=phi0, u0=u0, storage=storage, modes=modes, **TWO_PHASE)
    r0 = g.reduce()
    g.step(2)
    r1 = g.reduce()
    m = g.moments()
    zi, yi, xi = (torch.tensor([p[a] for p in pts], device="cuda") for a in range(3))
    gu = m["u"][:, zi, yi, xi].double().cpu().numpy()
    gphi = m["phi"][zi, yi, xi].double().cpu().numpy()
    g.close()
    del m, g
    gc.collect()
    torch.cuda.empty_cache()
    if extra_check is not None:
        extra_check(r0, r1)
    print(f"case largest box shape={shape} storage={storage}: oracle on {len(pts)} windows", flush=True)
    ou, ophi = [], []
    c = W // 2
    for p in pts:
        origin = tuple(int(v) - c for v in p)
        o = O.Oracle((W, W, W), tau, phi0=_window(phi0, origin, shape),
                     u0=np.stack([_window(u0[a], origin, shape) for a in range(3)]), **TWO_PHASE)
        o.set_accel(O.forcing_window(modes, shape, origin, (W, W, W)))
        o.step(2)
        mo = o.moments()
        ou.append(mo["u"][:, c, c, c])
        ophi.append(mo["phi"][c, c, c])
    ou, ophi = np.array(ou).T, np.array(ophi)
    e_max = float(np.abs(gu - ou).max() / np.abs(ou).max())
    print(f"sampled sites: u max |du| / max |u_o| {e_max:.3e}")
    return max(_relerr(gu, ou), e_max), float(np.abs(gphi - ophi).max())


def _points(phi0, shape, rng, n_iface=8):
    nz, ny, nx = shape
    sub = phi0[::2, ::4, ::4]
    iface = np.argwhere((sub > 0.1) & (sub < 0.9)) * np.array([2, 4, 4])
    pick = rng.choice(len(iface), min(n_iface, len(iface)), replace=False)
    pts = [tuple(int(v) for v in p) for p in iface[pick]]
    pts += [tuple(int(v) for v in rng.integers(0, (nz, ny, nx))) for _ in range(3)]
    # domain corners and work-item tile (64 x 4) boundaries, (z, y, x)
    pts += [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (nz - 1, ny - 1, 0), (0, ny - 1, nx - 1), (nz // 2, 3, 63),
            (nz // 2 - 1, 4, 64), (nz - 2, ny - 4, nx - 64), (1, ny // 2, nx // 2 - 1)]
    return pts


def _need(nbytes):
    import torch

    gc.collect()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes:
        pytest.skip(f"needs {nbytes / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} GiB free")


@pytest.mark.timeout(900)
def test_largest_plane_fp32_sampled_sites():
    from paper_2505_01126_amd import lbm

    shape = (8, 4096, 4096)
    cfg, _ = lbm.make_config(shape, 0.6, two_phase=True, storage="f32")
    _need(lbm.lbm_workspace_bytes(cfg) + 12 * 2**30)
    print(f"case largest plane shape={shape}: inputs", flush=True)
    phi0, _, _ = I.bubble_pack(shape, 64, 6.0, seed=67)
    u0 = I.random_u(shape, 0.02, seed=68)
    modes = I.forcing_modes(1e-5, seed=69)
    pts = _points(phi0, shape, np.random.default_rng(70))
    e_u, e_phi = _sampled_parity(shape, "f32", 0.6, phi0, u0, modes, pts)
    print(f"nx*ny = 2^24, FP32, {len(pts)} sites after 2 steps: u rel err (L2 or max) {e_u:.3e}, "
          f"phi max abs {e_phi:.3e}")
    assert e_u < 1e-5
    assert e_phi < 1e-5


@pytest.mark.timeout(900)
def test_largest_box_fp16_sampled_sites():
    from paper_2505_01126_amd import lbm

    shape = (64, 4096, 4096)
    cfg, _ = lbm.make_config(shape, 0.6, two_phase=True, storage="f16")
    _need(lbm.lbm_workspace_bytes(cfg) + 40 * 2**30)
    print(f"case largest box shape={shape}: inputs", flush=True)
    phi0, _, _ = I.bubble_pack(shape, 512, 16.0, seed=71)
    u0 = I.random_u(shape, 0.02, seed=72)
    modes = I.forcing_modes(1e-5, seed=73)
    pts = _points(phi0, shape, np.random.default_rng(74))
    sum_phi0 = float(np.sum(phi0))

    def conservation(r0, r1):
        print(f"sum phi: numpy {sum_phi0!r}, device t=0 {r0[0]!r}, t=2 {r1[0]!r}; non-finite sites {r1[9]}")
        assert abs(r0[0] - sum_phi0) < 1e-12 * sum_phi0
        assert abs(r1[0] - r0[0]) < 1e-12 * r0[0]
        assert r0[9] == 0 and r1[9] == 0

    e_u, e_phi = _sampled_parity(shape, "f16", 0.6, phi0, u0, modes, pts, conservation)
    print(f"nx*ny*nz = 2^30, FP16, {len(pts)} sites after 2 steps: u rel err (L2 or max) {e_u:.3e}, "
          f"phi max abs {e_phi:.3e}")
    assert e_u < 1e-3
    assert e_phi < 1e-4
