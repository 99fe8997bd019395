"""Learned-curvature network kernels (FP16 MFMA) against the FP64 oracle.

The oracle evaluates the same network with fp16 rounding of the inputs and of
the hidden activations; the GPU accumulates in FP32 inside the MFMA, so an
activation can land on the other side of an fp16 rounding boundary (one fp16
ulp, ~5e-4 relative).  Bars: forward outputs within 2e-3 of the output scale,
gradient relative L2 error below 1e-2 (the GPU backward runs its products on
fp16 operands), loss within 1e-3.  Batch sizes are ragged against the 16-sample
MFMA tile and the 64-sample workgroup chunk.
"""
import numpy as np
import pytest

import oracle as O
from parity import U_BAR, check
from paper_2505_01126_amd import inputs as I

pytestmark = pytest.mark.gpu
NP = O.MLP_NPARAM


def _lbm():
    from paper_2505_01126_amd import lbm

    return lbm


def _weights(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(NP) * scale
    return w.astype(np.float16).astype(np.float64)


def _inputs(B, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (B, 27)).astype(np.float16).astype(np.float64)
    xp = np.zeros((B, 32), dtype=np.float16)
    xp[:, :27] = x
    return x, xp


def _dev_x(xp):
    import torch

    return torch.tensor(xp.view(np.int16), device="cuda")


@pytest.mark.parametrize("B", [1, 37, 1000])
def test_forward_matches_oracle(B):
    import torch

    lbm = _lbm()
    w = _weights(1)
    x, xp = _inputs(B, 2)
    net = lbm.Mlp(w)
    y = net.forward(_dev_x(xp)).cpu().numpy().astype(np.float64)
    yo = O.mlp_forward(w, x)
    scale = np.abs(yo).max()
    err = np.abs(y - yo)
    print(f"forward B={B}: max err {err.max():.3e}, median {np.median(err):.3e}, scale {scale:.3f}")
    assert err.max() < 2e-3 * scale
    assert np.median(err) < 1e-4 * scale


@pytest.mark.parametrize("B", [50, 777])
def test_backward_matches_oracle(B):
    import torch

    lbm = _lbm()
    w = _weights(3)
    x, xp = _inputs(B, 4)
    t = np.random.default_rng(5).uniform(-1, 1, (B, 4))
    net = lbm.Mlp(w)
    g, loss = net.backward(_dev_x(xp), torch.tensor(t, dtype=torch.float32, device="cuda"))
    g = g.cpu().numpy().astype(np.float64)
    loss = float(loss.cpu().numpy()[0])
    lo, go = O.mlp_loss_grad(w, x, t.astype(np.float32).astype(np.float64))
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    print(f"backward B={B}: grad rel err {rel:.3e}, loss {loss:.6f} vs {lo:.6f}")
    assert rel < 1e-2
    assert loss == pytest.approx(lo, rel=1e-3)
    # every parameter block gets a gradient
    for a, b in ((0, 1728), (1728, 1792), (1792, 5888), (5888, 5952), (5952, 6208), (6208, 6212)):
        assert np.linalg.norm(g[a:b] - go[a:b]) <= 2e-2 * np.linalg.norm(go[a:b]) + 1e-7


def test_backward_deterministic_and_empty_batch():
    import torch

    lbm = _lbm()
    w = _weights(6)
    x, xp = _inputs(300, 7)
    t = torch.tensor(np.random.default_rng(8).uniform(-1, 1, (300, 4)), dtype=torch.float32, device="cuda")
    net = lbm.Mlp(w)
    g1 = net.backward(_dev_x(xp), t)[0].clone()
    g2 = net.backward(_dev_x(xp), t)[0].clone()
    assert torch.equal(g1, g2)
    y = net.forward(_dev_x(xp[:0]))
    assert y.shape == (0, 4)


def test_adam_matches_oracle():
    import torch

    lbm = _lbm()
    w = _weights(9)
    x, xp = _inputs(200, 10)
    t = np.random.default_rng(11).uniform(-1, 1, (200, 4))
    net = lbm.Mlp(w)
    wo = net.master.cpu().numpy().astype(np.float64)
    mo = np.zeros(NP)
    vo = np.zeros(NP)
    for step in range(1, 4):
        g, _ = net.backward(_dev_x(xp), torch.tensor(t, dtype=torch.float32, device="cuda"))
        gh = g.cpu().numpy().astype(np.float64)
        net.adam(lr=1e-3)
        w16o = O.adam(wo, mo, vo, gh, step, lr=1e-3)
    wm = net.master.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(wm, wo, rtol=1e-5, atol=1e-6)
    w16 = net.weights_fp16()
    assert np.mean(w16 == w16o) > 0.999


def test_harvest_matches_oracle():
    lbm = _lbm()
    shape = (24, 28, 70)
    phi, c, r = I.bubble_pack(shape, 3, (6.0, 10.0), seed=12)
    g = lbm.Lattice(shape, 0.8, phi0=phi, rho_l=1.0, rho_g=0.1, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)
    radii = -r  # phi = 0 inside
    X, Y, n = g.harvest(c, radii, cap=1 << 16)
    Xo, Yo, no = O.harvest(phi, c, radii)
    assert n == no == len(Xo)
    x16 = X.cpu().numpy().view(np.float16).astype(np.float64)
    np.testing.assert_array_equal(x16[:, :27], Xo.astype(np.float16).astype(np.float64))
    assert (x16[:, 27:] == 0).all()
    np.testing.assert_allclose(Y.cpu().numpy(), Yo, rtol=1e-6, atol=1e-7)
    # capacity smaller than the count: first rows only, total still reported
    X2, Y2, n2 = g.harvest(c, radii, cap=100)
    assert n2 == n and len(X2) == 100
    np.testing.assert_array_equal(X2.cpu().numpy(), X[:100].cpu().numpy())


def _mlp_case_weights(seed):
    """Weights whose normal output is near unit length for part of the inputs,
    so both the blended and the finite-difference fallback branches occur."""
    w = _weights(seed, scale=0.25)
    w[6208 + 1:6212] = [0.6, 0.5, 0.4]  # b3 for the normal outputs
    return w.astype(np.float16).astype(np.float64)


def test_step_with_learned_curvature_matches_oracle():
    import torch

    lbm = _lbm()
    shape = (24, 20, 70)
    phi_a, _ = I.droplet(shape, 3.0, 4.0, center=(20.3, 10.1, 12.2))
    phi_b, _ = I.droplet(shape, 4.0, 4.0, center=(52.7, 9.6, 11.4))
    phi0 = np.maximum(phi_a, phi_b)
    u0 = I.random_u(shape, 0.005, seed=31)
    w = _mlp_case_weights(32)
    kw = dict(rho_l=1.0, rho_g=0.1, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)
    g = lbm.Lattice(shape, 0.8, phi0=phi0, u0=u0, zchunk=8, curv_mode="mlp", **kw)
    with pytest.raises(lbm.LbmError):
        g.step(1)  # weights not installed yet
    g.set_mlp(torch.tensor(w.astype(np.float16).view(np.int16), device="cuda"))
    g.step(30)
    m = {k: v.double().cpu().numpy() for k, v in g.moments().items()}
    o = O.Oracle(shape, 0.8, phi0=phi0, u0=u0, curv_mode=1, mlp=w, **kw)
    o.step(30)
    mo = o.moments()
    # the learned force differs from the finite-difference one (the test is not vacuous)
    ofd = O.Oracle(shape, 0.8, phi0=phi0, u0=u0, **kw)
    ofd.step(30)
    mfd = ofd.moments()
    dfd = np.linalg.norm(mfd["u"] - mo["u"]) / np.linalg.norm(mo["u"])
    dfd_p = np.abs(mfd["p"] - mo["p"]).max() / np.abs(mo["p"] - mo["p"].mean()).max()
    # Both sides round the network's inputs, weights and hidden activations to
    # fp16 but form the sums in FP32 (MFMA) and FP64, so a rounding can land
    # one fp16 unit apart: the network's outputs differ by e_net (measured here
    # on the interface cells of the final field), and its share of the flow, dfd, responds
    # linearly to first order.  Bar: the FP32 bar of the finite-difference path
    # plus twice e_net times dfd; for the per-element p check, the largest
    # output difference times the network's share of the pressure variation.
    X, _, n = g.harvest(np.array([[20.3, 10.1, 12.2], [52.7, 9.6, 11.4]]), np.array([3.0, 4.0]), cap=1 << 16)
    y_gpu = lbm.Mlp(w).forward(X).double().cpu().numpy()
    y_orc = O.mlp_forward(w, X.cpu().numpy().view(np.float16)[:, :27].astype(np.float64))
    e_net = np.linalg.norm(y_gpu - y_orc) / np.linalg.norm(y_orc)
    e_net_max = np.abs(y_gpu - y_orc).max() / np.abs(y_orc).max()  # for the per-element p bar
    bar = 1e-5 + 2.0 * e_net * dfd
    p_bar = 1e-5 + 2.0 * e_net_max * dfd_p
    print(f"learned-curvature step: network outputs differ by {e_net:.3e} on {n} interface cells, FD vs learned "
          f"oracle runs by {dfd:.3e}; u bar {bar:.3e}")
    check(m, mo, "f32", "learned-curvature step", u_bar=bar, p_bar=p_bar, phi_bar=1e-5, drho=0.9)
    assert dfd > 1e-3 and n > 100


def test_learned_curvature_with_moving_interface_matches_oracle():
    """A droplet carried through small work items (z-chunks of 4 planes) by a
    uniform flow: its interface enters items that held none at the previous
    step, which the network pass must not skip (it skips items whose sites
    the previous step flagged as free of interface cells)."""
    import torch

    lbm = _lbm()
    shape = (40, 20, 24)
    phi0, c = I.droplet(shape, 4.0, 4.0, center=(11.6, 10.3, 12.8))
    u0 = np.zeros((3,) + shape)
    u0[2] = 0.04  # along z: 2.4 cells in 60 steps, across z-chunk boundaries
    w = _mlp_case_weights(33)
    kw = dict(rho_l=1.0, rho_g=1.0, sigma=0.005, mobility=0.05, width=4.0, p0=0.0)
    print("case moving droplet, learned curvature, zchunk 4", flush=True)
    g = lbm.Lattice(shape, 0.8, phi0=phi0, u0=u0, zchunk=4, curv_mode="mlp", **kw)
    g.set_mlp(torch.tensor(w.astype(np.float16).view(np.int16), device="cuda"))
    g.step(60)
    m = {k: v.double().cpu().numpy() for k, v in g.moments().items()}
    X, _, n = g.harvest(np.array([c]), np.array([4.0]), cap=1 << 16)
    y_gpu = lbm.Mlp(w).forward(X).double().cpu().numpy()
    g.close()
    y_orc = O.mlp_forward(w, X.cpu().numpy().view(np.float16)[:, :27].astype(np.float64))
    e_net = np.linalg.norm(y_gpu - y_orc) / np.linalg.norm(y_orc)
    e_net_max = np.abs(y_gpu - y_orc).max() / np.abs(y_orc).max()
    o = O.Oracle(shape, 0.8, phi0=phi0, u0=u0, curv_mode=1, mlp=w, **kw)
    o.step(60)
    mo = o.moments()
    ofd = O.Oracle(shape, 0.8, phi0=phi0, u0=u0, **kw)
    ofd.step(60)
    mfd = ofd.moments()
    dfd = np.linalg.norm(mfd["u"] - mo["u"]) / np.linalg.norm(mo["u"])
    dfd_p = np.abs(mfd["p"] - mo["p"]).max() / np.abs(mo["p"] - mo["p"].mean()).max()
    zc = [float((mo["phi"] * np.arange(shape[0])[:, None, None]).sum() / mo["phi"].sum())]
    print(f"moving droplet: centre z {c[2]:.2f} -> {zc[0]:.2f}; network outputs differ by {e_net:.3e} on {n} cells; "
          f"FD vs learned oracle runs by {dfd:.3e}")
    check(m, mo, "f32", "moving droplet, learned curvature", u_bar=1e-5 + 2.0 * e_net * dfd,
          p_bar=1e-5 + 2.0 * e_net_max * dfd_p, phi_bar=1e-5, drho=0.0)
    assert dfd > 1e-4 and zc[0] - c[2] > 2.0


def _learned_vs_oracle(lbm, shape, phi0, u0, w, kw, steps, label, storage="f32", **lattice_kw):
    """Run the learned-curvature step on the GPU and in the FP64 oracle; the
    bars as in test_step_with_learned_curvature_matches_oracle (the network
    output difference e_net times the network's share of the flow)."""
    import torch

    print(f"case {label}", flush=True)
    g = lbm.Lattice(shape, 0.8, phi0=phi0, u0=u0, curv_mode="mlp", storage=storage, **lattice_kw, **kw)
    g.set_mlp(torch.tensor(w.astype(np.float16).view(np.int16), device="cuda"))
    g.step(steps)
    m = {k: v.double().cpu().numpy() for k, v in g.moments().items()}
    ny, nx = shape[1], shape[2]
    X, _, n = g.harvest(np.array([[nx / 2.0, ny / 2.0, shape[0] / 2.0]]), np.array([4.0]), cap=1 << 16)
    y_gpu = lbm.Mlp(w).forward(X).double().cpu().numpy()
    g.close()
    y_orc = O.mlp_forward(w, X.cpu().numpy().view(np.float16)[:, :27].astype(np.float64))
    e_net = np.linalg.norm(y_gpu - y_orc) / np.linalg.norm(y_orc)
    e_net_max = np.abs(y_gpu - y_orc).max() / np.abs(y_orc).max()
    o = O.Oracle(shape, 0.8, phi0=phi0, u0=u0, curv_mode=1, mlp=w, **kw)
    o.step(steps)
    mo = o.moments()
    ofd = O.Oracle(shape, 0.8, phi0=phi0, u0=u0, **kw)
    ofd.step(steps)
    mfd = ofd.moments()
    dfd = np.linalg.norm(mfd["u"] - mo["u"]) / np.linalg.norm(mo["u"])
    dfd_p = np.abs(mfd["p"] - mo["p"]).max() / np.abs(mo["p"] - mo["p"].mean()).max()
    print(f"{label}: network outputs differ by {e_net:.3e} on {n} cells; FD vs learned oracle runs by {dfd:.3e}")
    ub = U_BAR[storage]
    check(m, mo, storage, label, u_bar=ub + 2.0 * e_net * dfd, p_bar=ub + 2.0 * e_net_max * dfd_p,
          phi_bar=ub, drho=kw["rho_l"] - kw["rho_g"])
    assert dfd > 1e-4 and n > 50


def test_learned_curvature_with_fixed_point_phi_matches_oracle():
    """The network pass and the learned step with the int32 fixed-point phase
    field (the pass stages phi converted from the fixed-point grid), against
    the FP64 oracle: the quantum 2^-30 is far below the bars."""
    lbm = _lbm()
    shape = (24, 20, 70)
    phi_a, _ = I.droplet(shape, 3.0, 4.0, center=(20.3, 10.1, 12.2))
    phi_b, _ = I.droplet(shape, 4.0, 4.0, center=(52.7, 9.6, 11.4))
    phi0 = np.maximum(phi_a, phi_b)
    u0 = I.random_u(shape, 0.005, seed=41)
    kw = dict(rho_l=1.0, rho_g=0.1, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)
    _learned_vs_oracle(lbm, shape, phi0, u0, _mlp_case_weights(34), kw, 30, "learned curvature, fix32 phi",
                       zchunk=8, phi_storage="fix32")


def test_learned_curvature_in_a_thin_box_with_ragged_z_chunks_matches_oracle():
    """A box eight planes thick (the smallest allowed) cut into z-chunks of
    3, 3 and 2 planes: the network pass stages planes z0-1 .. z0+3 ahead and
    runs its plane loop three planes at a time, so a chunk shorter than three
    planes, the periodic wrap of the staged planes and planes fetched past the
    chunk all occur.  The drop is a column along z, curved in x and y only."""
    lbm = _lbm()
    shape = (8, 24, 40)
    z, y, x = I.grid(shape)
    r = np.sqrt((x - 19.6) ** 2 + (y - 11.8) ** 2) + 0.0 * z
    phi0 = I.tanh_profile(4.0 - r, 4.0)
    u0 = I.random_u(shape, 0.005, seed=42)
    kw = dict(rho_l=1.0, rho_g=0.5, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)
    _learned_vs_oracle(lbm, shape, phi0, u0, _mlp_case_weights(35), kw, 40,
                       "learned curvature, nz = 8, z-chunks 3 3 2", zchunk=3)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_learned_curvature_with_16bit_populations_matches_oracle(storage):
    """The learned-curvature step with FP16 and BF16 population storage (the
    pass is the same; the step's 16-bit variants read its output), against
    the FP64 oracle at the storage's bars."""
    lbm = _lbm()
    shape = (24, 20, 70)
    phi_a, _ = I.droplet(shape, 3.0, 4.0, center=(20.3, 10.1, 12.2))
    phi_b, _ = I.droplet(shape, 4.0, 4.0, center=(52.7, 9.6, 11.4))
    phi0 = np.maximum(phi_a, phi_b)
    u0 = I.random_u(shape, 0.005, seed=43)
    kw = dict(rho_l=1.0, rho_g=0.1, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)
    _learned_vs_oracle(lbm, shape, phi0, u0, _mlp_case_weights(36), kw, 30, f"learned curvature, {storage} populations",
                       storage=storage, zchunk=8)
