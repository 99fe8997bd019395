"""Throughput of the fused lattice update on one MI355X.

Workload (default): 512^3 bubble-laden forced HIT, the bubbly-turbulence case
of Sec. 5.2 at the per-GPU size of the paper's weak-scaling runs (Sec. 4):
256 bubbles of diameter 16 at seeded non-overlapping positions, density ratio
10, sigma = 0.005, interface width 4, mobility 0.05, tau = 0.515 (nu = 0.005,
the paper's benchmark viscosity), large-scale forcing on the shells
0 < |k|^2 <= 4 with seeded phases, initial velocity a seeded solenoidal field of
rms 0.02.  Populations stored in FP32 (the reported value) and in FP16 / BF16
(reported beside it); arithmetic is FP32 in every variant.

A step is one fused kernel launch over the whole box.  Inputs are resident in
HBM before timing starts; W untimed warm-up steps, then K timed steps between
two stream synchronisations, timed with HIP events on the launch stream.

Prints one JSON line.  MLUPS = N * K / (t * 1e6).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# algorithmic bytes per lattice update: 27 population reads + 27 writes,
# phi FP64 read + write, u FP32 x3 read + write (the advecting velocity)
BYTES_PER_LUP = {"f32": 27 * 4 * 2 + 8 + 8 + 12 + 12, "f16": 27 * 2 * 2 + 40, "bf16": 27 * 2 * 2 + 40}
KERNEL_SOURCES = ["paper_2505_01126_amd/csrc/lbm_kernels.hip", "paper_2505_01126_amd/csrc/lbm_internal.h"]


def kernel_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def workload(n, seed=0):
    from paper_2505_01126_amd import inputs as I

    shape = (n, n, n)
    nb = max(1, int(round(256 * (n / 512.0) ** 3)))
    phi0, centers, radii = I.bubble_pack(shape, nb, 16.0, width=4.0, seed=seed)
    u0 = I.solenoidal_field(shape, rms=0.02, k0=4.0, seed=seed + 1)
    modes = I.forcing_modes(1e-5, seed=seed + 2)
    params = dict(rho_l=1.0, rho_g=0.1, sigma=0.005, mobility=0.05, width=4.0, p0=0.0, modes=modes)
    return shape, phi0, u0, params, nb


def traffic_for(workload_name, storage):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tab = json.load(f)
    rec = tab.get(f"{workload_name}:{storage}")
    if not rec or rec.get("kernel_sha") != kernel_sha():
        return None
    return rec.get("bytes_per_launch")


def time_variant(shape, phi0, u0, params, storage, steps, warmup, tau, zchunk):
    import torch

    from paper_2505_01126_amd import lbm

    g = lbm.Lattice(shape, tau, phi0=phi0, u0=u0, storage=storage, zchunk=zchunk, **params)
    r0 = g.reduce()
    stream = g.stream
    g.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    r1 = g.reduce()
    g.close()
    del g
    torch.cuda.empty_cache()
    return ms / steps, r0, r1


def cpu_baseline(seconds=15.0):
    """The FP64 oracle on a 64^3 box of the same recipe (one d = 16 bubble,
    same parameters and forcing), timed over whole steps until `seconds` pass."""
    import oracle as O

    shape, phi0, u0, params, nb = workload(64, seed=0)
    o = O.Oracle(shape, 0.515, phi0=phi0, u0=u0, **params)
    o.step(1)
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < seconds:
        o.step(2)
        steps += 2
    dt = time.perf_counter() - t0
    N = shape[0] * shape[1] * shape[2]
    return {"value": N * steps / dt / 1e6, "unit": "MLUPS", "cores": O.threads(), "kind": "oracle",
            "sample": f"64^3 box of the same recipe ({nb} bubble of d=16, same parameters and forcing), "
                      f"{steps} steps in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--storage", default="f32,f16,bf16")
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run 10 device-to-device copies of this many MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the z-slab multi-GPU layout is described in the design notes but not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_mib > 0:
        a = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 10
        print(json.dumps({"copy_mib": args.copy_mib, "copy_gbs": 2 * a.numel() / dt / 1e9}), flush=True)
        return
    t_setup = time.perf_counter()
    shape, phi0, u0, params, nb = workload(args.size)
    print(f"# inputs ready in {time.perf_counter() - t_setup:.1f} s: {args.size}^3, {nb} bubbles", file=sys.stderr,
          flush=True)
    N = shape[0] * shape[1] * shape[2]
    tau = 0.515
    name = f"bubbly_hit_{args.size}"
    variants = {}
    for st in [s.strip() for s in args.storage.split(",") if s.strip()]:
        ms, r0, r1 = time_variant(shape, phi0, u0, params, st, args.steps, args.warmup, tau, args.zchunk)
        mlups = N / (ms * 1e-3) / 1e6
        achieved = BYTES_PER_LUP[st] * N / (ms * 1e-3) / 1e9
        variants[st] = {
            "mlups": mlups, "ms_per_step": ms, "bytes_per_lup": BYTES_PER_LUP[st],
            "achieved_gbs": achieved, "frac": achieved / HBM_PEAK_GBS,
            "phase_volume_drift": abs(r1[0] - r0[0]) / r0[0], "nonfinite": int(r1[9]), "max_u": r1[7],
        }
        print(f"# {st}: {ms:.3f} ms/step, {mlups:.0f} MLUPS, {achieved:.0f} GB/s ({achieved / HBM_PEAK_GBS:.1%})",
              file=sys.stderr, flush=True)
    primary = "f32" if "f32" in variants else next(iter(variants))
    v = variants[primary]
    traffic = traffic_for(name, primary)
    line = {
        "metric": "MLUPS & % HBM roofline, 512^3 bubbly HIT, FP32 vs FP16-stored populations",
        "value": v["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": v["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "grid": list(shape), "bubbles": nb, "bubble_diameter": 16,
                   "density_ratio": 10, "sigma": 0.005, "tau": tau, "storage": primary,
                   "curvature": "fd", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": v["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": v["frac"], "traffic": traffic},
        "variants": variants,
        "kernel_sha": kernel_sha(),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
