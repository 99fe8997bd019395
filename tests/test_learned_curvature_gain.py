"""What the learned curvature gains over the finite-difference curvature.

The network (27 -> 64 -> 64 -> 4, FP16 MFMA training kernels) is trained with
train_curvature's default recipe: 96 periodic 48^3 boxes of 4 droplets or
bubbles with radii in [2, 10] (1/R uniform, so small spheres contribute as
many interface cells as large ones), relaxed by the coupled solver and
harvested with the Laplace-consistent curvature label K = (2 / R_eff) / I (I
the integral of the surface-tension profile across the relaxed sphere);
32000 Adam steps of 16384 rows drawn in proportion to |grad phi|^2 and turned by
random cube symmetries.  It is evaluated on spheres it has not seen:

1. the Laplace jump that the surface-tension force of Eq. (8) carries across
   each held-out relaxed sphere, (3 delta / 2) sigma sum K |grad phi|^2 /
   (4 pi r^2) over its interface cells, against 2 sigma / R_eff, with the
   network's K and with the finite-difference K (the oracle's FP64 curvature
   of the same field);
2. Laplace's law on droplets of R = 3, 4, 6 (diameters 6 to 12, the
   under-resolved range) relaxed for 1500 steps by the coupled solver with the
   learned blend on the ramp |K_FD| from 0.2 to 0.3, against the
   finite-difference run, at density ratio 1 and 10, with a bound on the
   spurious currents.  R = 2.5 is printed, not asserted: there the blend loses
   to finite differences at both density ratios;
3. the same at the benchmark's fluid (tau = 0.515, sigma = 0.005) with the
   library's ramp (0.4 to 0.6), 3000 steps, the pressure averaged over the
   last 200: the blend wins at R = 4 and 6, and at R = 3 for density ratio
   10.  R = 3 at ratio 1 is printed, not asserted (there it loses): per-cell
   errors of the network's K and normal make the surface-tension force
   partly solenoidal, and at this viscosity the currents that drives matter.

Parity of the kernels themselves is covered by test_gpu_mlp.py.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2505_01126_amd import inputs as I

pytestmark = pytest.mark.gpu
SIGMA = 0.01
K_LO, K_HI = 0.2, 0.3  # the blend ramp on |K_FD| (the library's default is 0.4 .. 0.6)
CAPILLARY_U = SIGMA / (1.0 * (1.0 - 0.5) / 3.0)  # sigma / (rho_l nu) at tau = 1


@pytest.fixture(scope="module")
def trained():
    from paper_2505_01126_amd import train_curvature as tc

    X, Y = tc.generate(seed=0, verbose=False)
    net, losses = tc.train(X, Y, seed=0, log_every=2000)
    print(f"training rows {X.shape[0]}, loss {losses[0][1]:.3e} -> {losses[-1][1]:.3e}")
    assert losses[-1][1] < 0.01 * losses[0][1]
    return net


def test_learned_curvature_carries_the_laplace_jump_of_unseen_spheres(trained):
    from paper_2505_01126_amd import train_curvature as tc

    rng = np.random.default_rng(1234)
    rows = []
    for bubbles in (False, True, False, True):
        g, phi, centers, signed = tc.relaxed_box(rng, 40, 3, 3.0, 7.0, 300, bubbles)
        X, _, n = g.harvest(centers, signed, cap=1 << 20)
        g.close()
        mask = (phi > 0.02) & (phi < 0.98)  # the harvested cells, in site order
        assert n == int(mask.sum())
        k_net = np.abs(trained.forward(X).double().cpu().numpy()[:, 0])
        k_fd = np.abs(O.curvature(phi)[0][mask])
        g2 = (O.gradient(phi) ** 2).sum(axis=0)[mask]
        owner, d2 = tc._owners(phi.shape, centers)
        owner, w = owner[mask], g2 / (4.0 * math.pi * np.maximum(d2[mask], 0.25))
        for k, r in enumerate(np.abs(signed)):
            sel = owner == k
            jump = lambda K: 1.5 * 4.0 * float((K[sel] * w[sel]).sum()) / (2.0 / r) - 1.0  # noqa: E731
            rows.append((r, jump(k_net), jump(k_fd)))
    rows = np.array(rows)
    for r, en, ef in rows:
        print(f"R_eff {r:.2f}: force-carried jump / (2 sigma / R_eff) - 1: network {en:+.4f}, FD {ef:+.4f}")
    e_net, e_fd = np.abs(rows[:, 1]).mean(), np.abs(rows[:, 2]).mean()
    print(f"{len(rows)} spheres: mean |error| network {e_net:.4f}, FD {e_fd:.4f}")
    assert e_net < 0.5 * e_fd


def _laplace(mode, R, ratio, w16, n=32, steps=1500, tau=1.0, sigma=SIGMA, ramp=(K_LO, K_HI), window=1):
    """Laplace error and max|u| after `steps`; with window > 1 the pressure is
    averaged over `window` snapshots 20 steps apart ending there (at low
    viscosity the pressure oscillates for thousands of steps)."""
    from paper_2505_01126_amd import lbm

    phi0, c = I.droplet((n, n, n), R, 4.0, seed=int(R * 10))
    print(f"case Laplace {mode} R={R} ratio={ratio} tau={tau} sigma={sigma} ramp={ramp}", flush=True)
    g = lbm.Lattice((n, n, n), tau, phi0=phi0, rho_l=1.0, rho_g=1.0 / ratio, sigma=sigma, mobility=0.05,
                    width=4.0, p0=0.0, curv_mode=mode, mlp_k_lo=ramp[0], mlp_k_hi=ramp[1])
    if mode == "mlp":
        g.set_mlp(w16)
    g.step(steps - 20 * (window - 1))
    ps, umax = [], 0.0
    for j in range(window):
        if j:
            g.step(20)
        m = {k: v.double().cpu().numpy() for k, v in g.moments().items()}
        ps.append(m["p"])
        umax = max(umax, float(np.abs(m["u"]).max()))
    g.close()
    phi, p = m["phi"], np.mean(ps, axis=0)
    reff = (3.0 * phi.sum() / (4.0 * math.pi)) ** (1.0 / 3.0)
    z, y, x = I.grid((n, n, n))
    d = np.sqrt(((x - c[0] + n / 2) % n - n / 2) ** 2 + ((y - c[1] + n / 2) % n - n / 2) ** 2 +
                ((z - c[2] + n / 2) % n - n / 2) ** 2)
    dp = p[d < 1.5].mean() - p[d > R + 12].mean()
    return dp / (2.0 * sigma / reff) - 1.0, umax


@pytest.mark.parametrize("ratio", [1.0, 10.0])
def test_learned_curvature_improves_laplace_law(trained, ratio):
    for R in (2.5, 3.0, 4.0, 6.0):
        efd, ufd = _laplace("fd", R, ratio, None)
        enet, unet = _laplace("mlp", R, ratio, trained.w16)
        print(f"ratio {ratio:g} R {R:g}: Laplace error FD {efd:+.4f} (max|u| {ufd:.1e}), "
              f"learned {enet:+.4f} (max|u| {unet:.1e}, {unet / ufd:.1f}x FD)")
        if R >= 3.0:
            assert abs(enet) < abs(efd)
        # spurious currents: bounded against the FD run and the capillary velocity
        assert unet < 25.0 * ufd and unet < 0.1 * CAPILLARY_U


@pytest.mark.parametrize("ratio", [1.0, 10.0])
def test_learned_curvature_at_low_viscosity(trained, ratio):
    for R in (3.0, 4.0, 6.0):
        kw = dict(steps=3000, tau=0.515, sigma=0.005, ramp=(0.4, 0.6), window=10)
        efd, ufd = _laplace("fd", R, ratio, None, **kw)
        enet, unet = _laplace("mlp", R, ratio, trained.w16, **kw)
        print(f"tau 0.515, ratio {ratio:g} R {R:g}: Laplace error FD {efd:+.4f} (max|u| {ufd:.1e}), "
              f"learned {enet:+.4f} (max|u| {unet:.1e}, {unet / ufd:.1f}x FD)")
        if R >= 4.0 or ratio == 10.0:
            assert abs(enet) < abs(efd)
