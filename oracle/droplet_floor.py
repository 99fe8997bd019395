"""How well-conditioned is the static-droplet velocity?  TEST INFRASTRUCTURE.

The velocity of a static droplet is its spurious current: the residue of the
surface-tension and pressure forces of Eq. (8), which cancel to within the
discretisation error at every interface cell.  This script runs the FP64
oracle on the static-droplet configuration (64^3, R 12, density ratio 10,
sigma 0.01, tau 1, 5000 steps) three times:

  * as it stands (the reference run);
  * from phi0 rounded once to FP32;
  * with the stored populations rounded to FP32 after every step, in the
    shifted form h_i = f_i / w_i - P0 that FP32 storage keeps.

and prints, for each perturbed run, the relative L2 difference of u against
the reference run and max |du| / max |u|, at several times.  The two
perturbed runs are the FP64 method itself, fed the rounding that FP32 storage
makes; their difference from the reference run is a floor under any FP32
implementation's distance from the oracle on this configuration.

Run: python -m oracle.droplet_floor [--steps 5000] [--size 64]
It calls only the oracle (and the seeded input generator).
"""
import argparse
import time

import numpy as np

from . import oracle as O


def _droplet(shape, radius, width, seed):
    from paper_2505_01126_amd import inputs as I  # seeded generator: no arithmetic of the method

    return I.droplet(shape, radius, width, seed=seed)[0]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--size", type=int, default=64)
    ap.add_argument("--every", type=int, default=1000)
    a = ap.parse_args()
    shape = (a.size,) * 3
    phi0 = _droplet(shape, 12.0, 4.0, 1)
    kw = dict(rho_l=1.0, rho_g=0.1, sigma=0.01, mobility=0.05, width=4.0, p0=0.0)
    _, w = O.lattice()
    wcol = w.reshape(27, 1, 1, 1)

    runs = {
        "reference": O.Oracle(shape, 1.0, phi0=phi0, **kw),
        "phi0 rounded to FP32 once": O.Oracle(shape, 1.0, phi0=phi0.astype(np.float32).astype(np.float64), **kw),
        "populations rounded to FP32 every step": O.Oracle(shape, 1.0, phi0=phi0, **kw),
    }
    per_step = runs["populations rounded to FP32 every step"]
    t0 = time.time()
    done = 0
    while done < a.steps:
        n = min(a.every, a.steps - done)
        runs["reference"].step(n)
        runs["phi0 rounded to FP32 once"].step(n)
        for _ in range(n):
            per_step.step(1)
            h = per_step.get_f() / wcol - kw["p0"]
            per_step.set_f((h.astype(np.float32).astype(np.float64) + kw["p0"]) * wcol)
        done += n
        uref = runs["reference"].moments()["u"]
        line = [f"step {done:5d} ({time.time() - t0:.0f} s): max |u| {np.abs(uref).max():.3e}"]
        for name, o in runs.items():
            if name == "reference":
                continue
            u = o.moments()["u"]
            rel = np.linalg.norm(u - uref) / np.linalg.norm(uref)
            mx = np.abs(u - uref).max() / np.abs(uref).max()
            line.append(f"  {name}: rel L2 {rel:.3e}, max|du|/max|u| {mx:.3e}")
        print("\n".join(line), flush=True)


if __name__ == "__main__":
    main()
