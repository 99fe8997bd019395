"""Train the learned-curvature network on droplets and bubbles the method generates.

Recipe (seeded): periodic boxes holding a few non-overlapping spheres of the
phi = 1 phase (droplets) or of the phi = 0 phase (bubbles) with radii drawn in
[r_min, r_max]; the coupled solver relaxes each box (static, density ratio 1,
tau = 1) so the interface takes the method's own discrete profile; interface
cells are harvested with the curvature label -2/R (droplet) or +2/R (bubble),
R the volume-equivalent radius of the relaxed sphere, and the radial normal.
Training runs the library's FP16 MFMA forward/backward and Adam kernels.

Usage: python -m paper_2505_01126_amd.train_curvature [--out weights.npy]
"""
from __future__ import annotations

import argparse
import math
import sys

import numpy as np

from . import inputs as I
from . import lbm

PARAMS = dict(rho_l=1.0, rho_g=1.0, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)


def _sphere_field(shape, centers, radii, width, bubbles):
    z, y, x = I.grid(shape)
    nz, ny, nx = shape
    sd = np.full(shape, np.inf)
    for c, r in zip(centers, radii):
        dx = x - c[0]
        dx -= nx * np.round(dx / nx)
        dy = y - c[1]
        dy -= ny * np.round(dy / ny)
        dz = z - c[2]
        dz -= nz * np.round(dz / nz)
        sd = np.minimum(sd, np.sqrt(dx * dx + dy * dy + dz * dz) - r)
    phi_in = I.tanh_profile(-sd, width)  # phi = 1 inside the spheres
    return 1.0 - phi_in if bubbles else phi_in


def _place(rng, box, per_box, r_min, r_max, width):
    centers, radii = [], []
    tries = 0
    while len(radii) < per_box and tries < 10000:
        tries += 1
        r = rng.uniform(r_min, r_max)
        c = rng.uniform(0, box, 3)
        ok = True
        for c2, r2 in zip(centers, radii):
            d = c - c2
            d -= box * np.round(d / box)
            if np.linalg.norm(d) < r + r2 + 3 * width:
                ok = False
                break
        if ok:
            centers.append(c)
            radii.append(r)
    return np.array(centers), np.array(radii)


def relaxed_box(rng, box, per_box, r_min, r_max, relax, bubbles, device="cuda:0"):
    """One periodic box of spheres relaxed by the coupled solver.  Returns the
    device Lattice (caller closes it), the FP64 phase field, the centres and
    the signed volume-equivalent radii (negative for bubbles)."""
    shape = (box, box, box)
    centers, radii = _place(rng, box, per_box, r_min, r_max, PARAMS["width"])
    phi0 = _sphere_field(shape, centers, radii, PARAMS["width"], bubbles)
    g = lbm.Lattice(shape, 1.0, phi0=phi0, device=device, **PARAMS)
    g.step(relax)
    phi = g.moments()["phi"].cpu().numpy()
    # volume-equivalent radius of each relaxed sphere (Voronoi by nearest centre)
    z, y, x = I.grid(shape)
    owner = np.zeros(shape, dtype=np.int64)
    best = np.full(shape, np.inf)
    for k, c in enumerate(centers):
        d2 = 0.0
        for a, coord in enumerate((x, y, z)):
            dd = coord - c[a]
            dd = dd - box * np.round(dd / box)
            d2 = d2 + dd * dd
        better = d2 < best
        owner = np.where(better, k, owner)
        best = np.where(better, d2, best)
    inside = (1.0 - phi) if bubbles else phi
    reff = np.array([(3.0 * float(inside[owner == k].sum()) / (4.0 * math.pi)) ** (1.0 / 3.0)
                     for k in range(len(centers))])
    return g, phi, centers, (-reff if bubbles else reff)


def generate(n_boxes=24, box=48, per_box=4, r_min=2.0, r_max=10.0, relax=300, seed=0, device="cuda:0",
             verbose=True):
    """Harvest training rows from relaxed method-generated spheres.
    Returns device tensors X [n, 32] (fp16 bits) and Y [n, 4] (FP32)."""
    import torch

    rng = np.random.default_rng(seed)
    Xs, Ys = [], []
    for b in range(n_boxes):
        bubbles = bool(b % 2)
        g, _, centers, signed = relaxed_box(rng, box, per_box, r_min, r_max, relax, bubbles, device)
        X, Y, n = g.harvest(centers, signed, cap=1 << 20)
        Xs.append(X.clone())
        Ys.append(Y.clone())
        g.close()
        if verbose:
            print(f"# box {b}: {'bubbles' if bubbles else 'droplets'} R={np.round(np.abs(signed), 2).tolist()} "
                  f"-> {n} rows", file=sys.stderr, flush=True)
    return torch.cat(Xs), torch.cat(Ys)


def init_weights(seed=0):
    """Xavier-uniform weights, zero biases, fp16-exact."""
    rng = np.random.default_rng(seed)
    w = np.zeros(lbm.MLP_NPARAM)
    o = 0
    for fan_out, fan_in in ((64, 27), (64, 64), (4, 64)):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        w[o:o + fan_out * fan_in] = rng.uniform(-lim, lim, fan_out * fan_in)
        o += fan_out * fan_in + fan_out
    return w.astype(np.float16).astype(np.float64)


def train(X, Y, steps=3000, batch=4096, lr=2e-3, seed=0, device="cuda:0", log_every=500):
    """Adam on minibatches drawn with a seeded generator; returns (Mlp, losses)."""
    import torch

    net = lbm.Mlp(init_weights(seed), device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    n = X.shape[0]
    losses = []
    for it in range(1, steps + 1):
        idx = torch.randint(0, n, (min(batch, n),), device=device, generator=gen)
        _, loss = net.backward(X[idx].contiguous(), Y[idx].contiguous())
        step_lr = lr * (0.5 * (1.0 + math.cos(math.pi * it / steps)))  # cosine decay
        net.adam(lr=step_lr)
        if it % log_every == 0 or it == 1:
            losses.append((it, float(loss.item())))
            print(f"# step {it}: loss {losses[-1][1]:.3e}", file=sys.stderr, flush=True)
    return net, losses


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="curvature_mlp.npy")
    ap.add_argument("--boxes", type=int, default=24)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args()
    X, Y = generate(n_boxes=a.boxes, seed=a.seed)
    net, losses = train(X, Y, steps=a.steps, seed=a.seed)
    np.save(a.out, net.weights_fp16())
    print(f"saved {a.out}; final loss {losses[-1][1]:.3e}")


if __name__ == "__main__":
    main()
