"""Throughput of the fused lattice update on one MI355X.

Workload (default): 512^3 bubble-laden forced HIT, the bubbly-turbulence case
of Sec. 5.2 at the per-GPU size of the paper's weak-scaling runs (Sec. 4):
256 bubbles of diameter 16 at seeded non-overlapping positions, density ratio
10, sigma = 0.005, interface width 4, mobility 0.05, tau = 0.515 (nu = 0.005,
the paper's benchmark viscosity), large-scale forcing on the shells
0 < |k|^2 <= 4 with seeded phases, initial velocity a seeded solenoidal field of
rms 0.02.  Populations stored in FP32 (the reported value) and in FP16 / BF16
(reported beside it); arithmetic is FP32 in every variant.  The phase field
is stored in FP64, or in int32 fixed point in the ":fix32" variants (4 bytes
less read and written per site).  The ":rk3" variants advance the phase field
with three Runge-Kutta stages: the step kernel's own update is the first, two
phase-field launches per step add the others.

A step is one fused kernel launch over the whole box (three launches with ":rk3").  Inputs are resident in
HBM before timing starts; W untimed warm-up steps, then R blocks of K timed
steps, each between two stream synchronisations and timed with HIP events on
the launch stream; the median block is reported.  The learned-curvature
variants run the same workload with the network blend switched on, with the
network that train_curvature trains (paper_2505_01126_amd/curvature_mlp.npy).

The small-bubble leg times the same recipe with 256 bubbles of d = 4..6 and
reports Laplace's law on those bubbles at rest (no velocity, no forcing) after
1000 steps: finite differences against the trained network's blend.

Each variant also reports its error against the FP64 oracle on a 64^3 box of
the same recipe after 50 steps (relative L2 of u, max |phi| difference).
cpu_baseline times that oracle on the host cores on the benchmark workload
itself (two steps after an untimed one), or on a 64^3 box of the recipe when
the host lacks memory for the 512^3 FP64 state.

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
PHI_BYTES_SAVED = {"f64": 0, "fix32": 4 + 4}  # int32 phi: 4 B read + 4 B written instead of 8 + 8
# each extra Runge-Kutta stage of phi: stage input and phi^n read, stage output
# written (FP64), the three face velocities read
RK3_STAGE_BYTES = 8 + 8 + 8 + 12


def parse_variant(key):
    """'storage[:curvature][:phi storage][:rk3]' -> (storage, curvature, phi storage, rk3)."""
    parts = key.split(":")
    st, curv, phs, rk3 = parts[0], "fd", "f64", False
    for p in parts[1:]:
        if p in ("fd", "mlp"):
            curv = p
        elif p in PHI_BYTES_SAVED:
            phs = p
        elif p == "rk3":
            rk3 = True
        else:
            raise SystemExit(f"bench.py: unknown variant field {p!r} in {key!r}")
    return st, curv, phs, rk3


def bytes_per_lup(st, phs="f64", rk3=False):
    return BYTES_PER_LUP[st] - PHI_BYTES_SAVED[phs] + (2 * RK3_STAGE_BYTES if rk3 else 0)
KERNEL_SOURCES = ["paper_2505_01126_amd/csrc/lbm_step.h", "paper_2505_01126_amd/csrc/lbm_step_s0.hip",
                  "paper_2505_01126_amd/csrc/lbm_step_s1.hip", "paper_2505_01126_amd/csrc/lbm_step_s2.hip",
                  "paper_2505_01126_amd/csrc/lbm_kernels.hip", "paper_2505_01126_amd/csrc/lbm_internal.h"]


def kernel_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


TWO_PHASE = dict(rho_l=1.0, rho_g=0.1, sigma=0.005, mobility=0.05, width=4.0, p0=0.0)
WEIGHTS = os.path.join(ROOT, "paper_2505_01126_amd", "curvature_mlp.npy")


def bubbles(n, seed=0, diameter=16.0):
    """The seeded bubble field of the recipe on n^3 (256 bubbles at 512^3, the
    same number density at other sizes): (shape, phi0, centres, radii, count)."""
    from paper_2505_01126_amd import inputs as I

    shape = (n, n, n)
    nb = max(1, int(round(256 * (n / 512.0) ** 3)))
    phi0, centers, radii = I.bubble_pack(shape, nb, diameter, width=4.0, seed=seed)
    return shape, phi0, centers, radii, nb


def workload(n, seed=0, diameter=16.0):
    """The bubbly-HIT recipe on n^3; `diameter` is a number or a (lo, hi)
    range sampled per bubble (the small-bubble run uses (4, 6))."""
    from paper_2505_01126_amd import inputs as I

    shape, phi0, _, _, nb = bubbles(n, seed, diameter)
    u0 = I.solenoidal_field(shape, rms=0.02, k0=4.0, seed=seed + 1)
    modes = I.forcing_modes(1e-5, seed=seed + 2)
    return shape, phi0, u0, dict(TWO_PHASE, modes=modes), nb


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


def trained_weights(path=WEIGHTS):
    """The network trained by train_curvature (seed 0, its default recipe), as
    a device tensor of fp16 bits."""
    import torch

    w = np.load(path, allow_pickle=False)
    if w.size != 6212:
        raise SystemExit(f"bench.py: {path} holds {w.size} values, not the network's 6212")
    return torch.tensor(w.astype(np.float16).view(np.int16).reshape(-1), device="cuda")


def mlp_weights(seed=5):
    """Seeded network weights (FP64 holding fp16 values) whose normal outputs
    are near unit length, so the blend branch of the step runs."""
    from paper_2505_01126_amd import lbm

    w = np.random.default_rng(seed).standard_normal(lbm.MLP_NPARAM) * 0.25
    w[-3:] = [0.6, 0.5, 0.4]
    return w.astype(np.float16).astype(np.float64)


def time_variant(shape, phi0, u0, params, storage, steps, warmup, repeats, tau, zchunk, curv="fd", phs="f64",
                 rk3=False):
    import torch

    from paper_2505_01126_amd import lbm

    g = lbm.Lattice(shape, tau, phi0=phi0, u0=u0, storage=storage, zchunk=zchunk, curv_mode=curv, phi_storage=phs,
                    ac_rk3=rk3, **params)
    if curv == "mlp":
        g.set_mlp(trained_weights())
    r0 = g.reduce()
    stream = g.stream
    g.step(warmup)
    torch.cuda.synchronize()
    times = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / steps)
    r1 = g.reduce()
    g.close()
    del g
    torch.cuda.empty_cache()
    return float(np.median(times)), r0, r1


def batch_leg(steps, warmup, repeats, count=128, seed=3):
    """Ensemble of `count` seeded bubble-in-box instances (edges 32..96, 1-8
    bubbles of d 6-20, density ratio 1-10; FP16 populations, learned curvature
    with finite-difference fallback; tau = 1, sigma = 0.01, at rest): aggregate
    MLUPS of one launch per instance per step vs one persistent batched launch
    per step (graph-replayed, z-chunk from the autotuner)."""
    import torch

    from paper_2505_01126_amd import inputs as I
    from paper_2505_01126_amd import lbm

    t0 = time.perf_counter()
    ens = I.bubble_box_ensemble(count, seed=seed)
    w16 = torch.tensor(mlp_weights().astype(np.float16).view(np.int16), device="cuda")
    gs = []
    for e in ens:
        g = lbm.Lattice(e["shape"], 1.0, phi0=e["phi0"], rho_l=1.0, rho_g=1.0 / e["ratio"], sigma=0.01,
                        mobility=0.05, width=4.0, p0=0.0, storage="f16", curv_mode="mlp")
        g.set_mlp(w16)
        gs.append(g)
    sites = sum(g.N for g in gs)
    print(f"# batch of {count} boxes ready in {time.perf_counter() - t0:.1f} s ({sites / 1e6:.1f} M sites)",
          file=sys.stderr, flush=True)
    stream = gs[0].stream

    def timed(run):
        times = []
        for _ in range(repeats):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run()
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / steps)
        return float(np.median(times))

    def per_instance(k):
        for _ in range(k):
            for g in gs:
                g.step(1)

    per_instance(warmup)
    ms_single = timed(lambda: per_instance(steps))
    b = lbm.Batch(gs)
    tile, zc = b.tune(2)
    b.step(warmup)
    ms_batch = timed(lambda: b.step(steps))
    b.close()
    for g in gs:
        g.close()
    del gs
    torch.cuda.empty_cache()
    return {"instances": count, "sites": sites, "storage": "f16", "curvature": "mlp", "tile": tile, "zchunk": zc,
            "ms_per_step_batched": ms_batch, "ms_per_step_per_instance": ms_single,
            "mlups_batched": sites / (ms_batch * 1e-3) / 1e6, "mlups_per_instance": sites / (ms_single * 1e-3) / 1e6,
            "speedup": ms_single / ms_batch}


def bubble_laplace(n=512, seed=0, diameter=(4.0, 6.0), curv="fd", w16=None, k_lo=0.0, k_hi=0.0,
                   checkpoints=(1000,), window=10):
    """Laplace's law on the bubbles of the recipe, at rest: no initial
    velocity and no forcing, FP32 populations, tau = 0.515, density ratio 10.
    At each checkpoint (steps from the start), per bubble whose nearest
    neighbour centre is at least 2 window + 2 away: R_eff from the gas volume
    sum (1 - phi) within `window` of its centre, dp = mean p within 1 of the
    centre - mean p at 8..10, and e = dp / (2 sigma / R_eff) - 1.  Returns,
    per checkpoint, the mean and mean |e| over those bubbles, the largest
    |e|, the R_eff range and the spurious currents: the largest |u| within
    `window` of the measured bubbles' centres, and max |u_a| over the box
    (which also sees closer pairs of bubbles)."""
    import torch

    from paper_2505_01126_amd import lbm

    shape, phi0, centers, radii, nb = bubbles(n, seed, diameter)
    L = float(n)
    dc = centers[:, None, :] - centers[None, :, :]
    dc -= L * np.round(dc / L)
    dist = np.sqrt((dc * dc).sum(-1)) + np.eye(nb) * 1e9
    keep = np.nonzero(dist.min(1) >= 2 * window + 2)[0]
    dev = torch.device("cuda")
    o = torch.arange(-window, window + 1, device=dev)
    oz, oy, ox = [t.reshape(-1) for t in torch.meshgrid(o, o, o, indexing="ij")]
    c = torch.tensor(centers[keep], device=dev, dtype=torch.float64)
    ci = torch.round(c).long()
    X, Y, Z = [(ci[:, a, None] + off) % n for a, off in ((0, ox), (1, oy), (2, oz))]
    idx = (Z * n + Y) * n + X
    d2 = 0.0
    for a, coord in enumerate((X, Y, Z)):
        dd = coord.double() - c[:, a, None]
        dd -= L * torch.round(dd / L)
        d2 = d2 + dd * dd
    d = torch.sqrt(d2)
    ball, core, shell = d <= window, d <= 1.0, (d >= 8.0) & (d <= 10.0)
    g = lbm.Lattice(shape, 0.515, phi0=phi0, storage="f32", curv_mode=curv, mlp_k_lo=k_lo, mlp_k_hi=k_hi,
                    **TWO_PHASE)
    if curv == "mlp":
        g.set_mlp(w16)
    out, done = [], 0
    for cp in checkpoints:
        g.step(cp - done)
        done = cp
        m = g.moments()
        phi = m["phi"].reshape(-1)[idx]
        p = m["p"].reshape(-1)[idx].double()
        reff = (3.0 * ((1.0 - phi) * ball).sum(1) / (4.0 * math.pi)).clamp(min=0.0) ** (1.0 / 3.0)
        dp = (p * core).sum(1) / core.sum(1) - (p * shell).sum(1) / shell.sum(1)
        e = (dp / (2.0 * TWO_PHASE["sigma"] / reff.clamp(min=1e-3)) - 1.0).cpu().numpy()
        r = reff.cpu().numpy()
        umag = torch.sqrt((m["u"].reshape(3, -1)[:, idx] ** 2).sum(0))
        out.append({"steps": cp, "bubbles_measured": int(len(keep)), "mean_err": float(e.mean()),
                    "mean_abs_err": float(np.abs(e).mean()), "max_abs_err": float(np.abs(e).max()),
                    "r_eff_min": float(r.min()), "r_eff_max": float(r.max()),
                    "max_u_measured": float(umag[ball].max()), "max_u": float(m["u"].abs().max()),
                    "nonfinite": int(g.reduce()[9])})
        del m
    g.close()
    del g
    torch.cuda.empty_cache()
    return out


def small_bubble_leg(steps, warmup, repeats, n=512, accuracy_steps=1000):
    """The same workload with 256 bubbles of d in [4, 6] (seeded): a step costs
    the same bytes, but far more cells take the learned-curvature branch.
    Beside the timings: Laplace's law on these bubbles at rest, finite
    differences against the trained network's blend (bubble_laplace)."""
    shape, phi0, u0, params, nb = workload(n, seed=0, diameter=(4.0, 6.0))
    N = shape[0] * shape[1] * shape[2]
    out = {"bubbles": nb, "diameter": [4.0, 6.0], "interface_cells": int(((phi0 > 0.02) & (phi0 < 0.98)).sum())}
    for key in ("f32", "f32:mlp", "f16:mlp"):
        st, curv, phs, rk3 = parse_variant(key)
        ms, r0, r1 = time_variant(shape, phi0, u0, params, st, steps, warmup, repeats, 0.515, 0, curv, phs, rk3)
        out[key] = {"ms_per_step": ms, "mlups": N / (ms * 1e-3) / 1e6, "nonfinite": int(r1[9])}
        print(f"# small bubbles {key}: {ms:.3f} ms/step", file=sys.stderr, flush=True)
    del phi0, u0
    if accuracy_steps > 0:
        acc = {}
        w16 = trained_weights()
        for name, kw in (("fd", {}), ("mlp", {"curv": "mlp", "w16": w16}),
                         ("mlp_ramp_0.2_0.3", {"curv": "mlp", "w16": w16, "k_lo": 0.2, "k_hi": 0.3})):
            acc[name] = bubble_laplace(n, checkpoints=(accuracy_steps,), **kw)[-1]
            a = acc[name]
            print(f"# small bubbles at rest, {name}, {accuracy_steps} steps: Laplace error mean {a['mean_err']:+.3f}, "
                  f"mean |e| {a['mean_abs_err']:.3f} over {a['bubbles_measured']} bubbles, max|u| {a['max_u_measured']:.2e} "
                  f"near them ({a['max_u']:.2e} in the box)",
                  file=sys.stderr, flush=True)
        out["laplace_at_rest"] = acc
    return out


def _spectrum(u):
    """Shell-summed kinetic energy spectrum E(k), k = 0 .. n/2, of a periodic
    field u [3, n, n, n] (torch, on the GPU): sum_k E(k) = <|u|^2> / 2."""
    import torch

    n = u.shape[-1]
    uh = torch.fft.rfftn(u.double(), dim=(1, 2, 3)) / n ** 3
    e = 0.5 * (uh.real ** 2 + uh.imag ** 2).sum(0)
    w = torch.full((n,), 2.0, dtype=torch.float64, device=u.device)[: n // 2 + 1]
    w[0] = 1.0
    w[-1] = 1.0  # the Nyquist plane of the half spectrum is not mirrored
    e = e * w
    k = torch.fft.fftfreq(n, 1.0 / n).to(u.device)
    kr = torch.fft.rfftfreq(n, 1.0 / n).to(u.device)
    kk = torch.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + kr[None, None, :] ** 2)
    shell = torch.round(kk).long().clamp(max=n // 2)
    return torch.zeros(n // 2 + 1, dtype=torch.float64, device=u.device).index_add_(0, shell.flatten(),
                                                                                     e.flatten())


def hit_report(steps=20000, every=2000, n=256, oracle_n=64, oracle_checks=(250, 500, 1000, 2000)):
    """Forced single-phase HIT (tau 0.55, solenoidal u0 of rms 0.02, forcing
    on 0 < |k|^2 <= 4): on n^3 for `steps` steps in FP32, FP16 and BF16
    population storage, the energy spectrum and the velocity difference from
    the FP32 run every `every` steps; on oracle_n^3, the velocity error of the
    three storages against the FP64 oracle at `oracle_checks` steps."""
    import torch

    import oracle as O
    from paper_2505_01126_amd import inputs as I
    from paper_2505_01126_amd import lbm

    out = {"n": n, "steps": steps, "tau": 0.55, "storage": {}, "oracle": {"n": oracle_n, "checks": {}}}
    shape = (n, n, n)
    u0 = I.solenoidal_field(shape, rms=0.02, k0=4.0, seed=1)
    modes = I.forcing_modes(1e-5, seed=2)
    ref = {}
    for st in ("f32", "f16", "bf16"):
        g = lbm.Lattice(shape, 0.55, u0=u0, modes=modes, p0=1.0, storage=st)
        rec = out["storage"][st] = {"step": [], "u_rms": [], "rel_diff_vs_f32": [], "spectrum": {}}
        done = 0
        while done < steps:
            g.step(every)
            done += every
            u = g.moments()["u"]
            rms = float(torch.sqrt((u.double() ** 2).sum(0).mean() / 3.0))
            if st == "f32":
                ref[done] = u.clone()
                diff = 0.0
            else:
                diff = float(torch.linalg.vector_norm((u - ref[done]).double())
                             / torch.linalg.vector_norm(ref[done].double()))
            rec["step"].append(done)
            rec["u_rms"].append(rms)
            rec["rel_diff_vs_f32"].append(diff)
            if done in (every, steps // 2, steps):
                rec["spectrum"][str(done)] = _spectrum(u).cpu().tolist()
            print(f"# HIT {n}^3 {st}: {done} steps, u_rms {rms:.5f}, vs f32 {diff:.2e}", file=sys.stderr,
                  flush=True)
        g.close()
    del ref
    torch.cuda.empty_cache()
    shape = (oracle_n,) * 3
    u0 = I.solenoidal_field(shape, rms=0.02, k0=4.0, seed=1)
    o = O.Oracle(shape, 0.55, u0=u0, modes=modes, p0=1.0)
    gs = {st: lbm.Lattice(shape, 0.55, u0=u0, modes=modes, p0=1.0, storage=st) for st in ("f32", "f16", "bf16")}
    done = 0
    for c in oracle_checks:
        o.step(c - done)
        for g in gs.values():
            g.step(c - done)
        done = c
        uo = o.moments()["u"]
        row = {}
        for st, g in gs.items():
            u = g.moments()["u"].double().cpu().numpy()
            row[st] = float(np.linalg.norm(u - uo) / np.linalg.norm(uo))
        out["oracle"]["checks"][str(c)] = row
        print(f"# HIT {oracle_n}^3 vs oracle at {c} steps: {row}", file=sys.stderr, flush=True)
    for g in gs.values():
        g.close()
    return out


def oracle_timing():
    """The FP64 oracle on the host cores for the four benchmark workloads:
    TGV 32^3 (200 steps), static droplet 64^3 (R = 12, ratio 10, all 5000
    steps of the configuration), single-phase forced HIT 256^3 (100 steps),
    512^3 bubbly HIT (3 blocks of 10 steps, median).  Each after one untimed
    step; prints a line per block of steps as it goes and returns MLUPS per
    workload."""
    import oracle as O
    from paper_2505_01126_amd import inputs as I

    out = {}

    def run(name, o, steps, chunk, repeats=1):
        o.step(1)
        blocks = []
        for r in range(repeats):
            t0 = time.perf_counter()
            done = 0
            while done < steps:
                k = min(chunk, steps - done)
                o.step(k)
                done += k
                print(f"# oracle {name} (block {r + 1}/{repeats}): {done}/{steps} steps, "
                      f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
            blocks.append(time.perf_counter() - t0)
        dt = float(np.median(blocks))
        out[name] = {"mlups": o.N * steps / dt / 1e6, "steps": steps, "seconds": dt, "blocks": len(blocks),
                     "block_seconds": blocks}

    u, p, _ = I.tgv((32, 32, 32), 0.02)
    run("tgv_32", O.Oracle((32, 32, 32), 0.8, u0=u, pstar0=p), 200, 100)
    phi0, _ = I.droplet((64, 64, 64), 12.0, 4.0, seed=1)
    run("droplet_64", O.Oracle((64, 64, 64), 1.0, phi0=phi0, rho_l=1.0, rho_g=0.1, sigma=0.01, mobility=0.05,
                               width=4.0, p0=0.0), 5000, 250)
    shape = (256, 256, 256)
    u0 = I.solenoidal_field(shape, rms=0.02, k0=4.0, seed=1)
    run("hit_256", O.Oracle(shape, 0.55, u0=u0, modes=I.forcing_modes(1e-5, seed=2)), 100, 5)
    del u0
    shape, phi0, u0, params, nb = workload(512)
    run("bubbly_hit_512", O.Oracle(shape, 0.515, phi0=phi0, u0=u0, **params), 10, 1, repeats=3)
    return {"cores": O.threads(), "nproc": os.cpu_count(), "workloads": out}


def copy_gbs(mib=1024, reps=10):
    """Device-to-device copy bandwidth (read + write bytes) on this GPU."""
    import torch

    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * (mib << 20) / dt / 1e9


def error_vs_oracle(storage, curv, phs="f64", rk3=False, steps=50, n=64):
    """Relative L2 error of u (and max |phi| difference) against the FP64
    oracle after `steps` steps on an n^3 box of the bench recipe."""
    import oracle as O
    from paper_2505_01126_amd import lbm
    import torch

    shape, phi0, u0, params, nb = workload(n, seed=0)
    g = lbm.Lattice(shape, 0.515, phi0=phi0, u0=u0, storage=storage, curv_mode=curv, phi_storage=phs, ac_rk3=rk3,
                    **params)
    w = None
    if curv == "mlp":
        w = mlp_weights()
        g.set_mlp(torch.tensor(w.astype(np.float16).view(np.int16), device="cuda"))
    g.step(steps)
    m = {k: v.double().cpu().numpy() for k, v in g.moments().items()}
    g.close()
    o = O.Oracle(shape, 0.515, phi0=phi0, u0=u0, curv_mode=1 if curv == "mlp" else 0, mlp=w, ac_rk3=rk3, **params)
    o.step(steps)
    mo = o.moments()
    return {"u_rel_l2": float(np.linalg.norm(m["u"] - mo["u"]) / np.linalg.norm(mo["u"])),
            "phi_max_abs": float(np.abs(m["phi"] - mo["phi"]).max()), "box": n, "steps": steps}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        return ""


def _mem_available_gib():
    try:
        with open("/proc/meminfo") as f:
            for ln in f:
                if ln.startswith("MemAvailable:"):
                    return int(ln.split()[1]) / 2 ** 20
    except OSError:
        pass
    return 0.0


def cpu_baseline(shape, phi0, u0, params, nb, steps=2, proxy_seconds=15.0):
    """The FP64 oracle on the host cores.  On the benchmark workload itself
    (the same seeded 512^3 fields and parameters) when the host has memory for
    its FP64 state (~62 GiB at 512^3): one untimed step, then `steps` timed
    steps, a bounded sample of about 25 s.  Otherwise a 64^3 box of the same
    recipe, timed over whole steps for `proxy_seconds`."""
    import oracle as O

    N = shape[0] * shape[1] * shape[2]
    need_gib = N * (2 * 27 + 12) * 8 / 2 ** 30 + 4
    out = {"unit": "MLUPS", "kind": "oracle", "cpu_model": _cpu_model(), "nproc": os.cpu_count()}
    if _mem_available_gib() > need_gib:
        t_init = time.perf_counter()
        o = O.Oracle(shape, 0.515, phi0=phi0, u0=u0, **params)
        o.step(1)
        t_init = time.perf_counter() - t_init
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
        del o
        out.update(value=N * steps / dt / 1e6, cores=O.threads(),
                   sample=f"the benchmark workload itself ({shape[0]}^3, {nb} bubbles of d=16): {steps} steps in "
                          f"{dt:.1f} s after one untimed step (set-up and that step {t_init:.1f} s)")
        return out
    shape, phi0, u0, params, nb = workload(64, seed=0)
    o = O.Oracle(shape, 0.515, phi0=phi0, u0=u0, **params)
    o.step(1)
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < proxy_seconds:
        o.step(2)
        done += 2
    dt = time.perf_counter() - t0
    n = shape[0] * shape[1] * shape[2]
    out.update(value=n * done / dt / 1e6, cores=O.threads(),
               sample=f"64^3 box of the same recipe ({nb} bubble of d=16, same parameters and forcing; the host "
                      f"had {_mem_available_gib():.0f} GiB free, under the {need_gib:.0f} GiB of the full "
                      f"workload), {done} steps in {dt:.1f} s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--repeats", type=int, default=5)
    ap.add_argument("--storage", default="f32,f16,bf16,f32:mlp,f16:mlp,f32:fix32,f16:fix32,f32:rk3,f16:rk3",
                    help="comma list of storage[:curvature][:phi storage][:rk3] variants (curvature fd|mlp, phi "
                         "f64|fix32, rk3: Runge-Kutta phase field); the first is the reported value")
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=2,
                    help="oracle steps timed on the benchmark workload for cpu_baseline (after one untimed step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 128-box ensemble leg")
    ap.add_argument("--no-small-bubbles", action="store_true", help="skip the d = 4..6 bubble leg")
    ap.add_argument("--hit-report", action="store_true",
                    help="only run the forced-HIT storage report (256^3 spectra over 20 000 steps, 64^3 error "
                         "against the oracle over time) and exit")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="only time the FP64 oracle on the four workloads (several minutes of CPU) and exit")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run 10 device-to-device copies of this many MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(there is no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    if args.oracle_timing:
        res = oracle_timing()
        res["cpu_model"] = _cpu_model()
        print(json.dumps(res), flush=True)
        return

    import torch

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.hit_report:
        print(json.dumps(hit_report()), flush=True)
        return
    if args.copy_mib > 0:
        print(json.dumps({"copy_mib": args.copy_mib, "copy_gbs": copy_gbs(args.copy_mib)}), flush=True)
        return
    t_setup = time.perf_counter()
    shape, phi0, u0, params, nb = workload(args.size)
    print(f"# inputs ready in {time.perf_counter() - t_setup:.1f} s: {args.size}^3, {nb} bubbles", file=sys.stderr,
          flush=True)
    N = shape[0] * shape[1] * shape[2]
    tau = 0.515
    name = f"bubbly_hit_{args.size}"
    variants = {}
    for key in [s.strip() for s in args.storage.split(",") if s.strip()]:
        st, curv, phs, rk3 = parse_variant(key)
        ms, r0, r1 = time_variant(shape, phi0, u0, params, st, args.steps, args.warmup, args.repeats, tau,
                                  args.zchunk, curv, phs, rk3)
        mlups = N / (ms * 1e-3) / 1e6
        blup = bytes_per_lup(st, phs, rk3)
        achieved = blup * N / (ms * 1e-3) / 1e9
        variants[key] = {
            "storage": st, "curvature": curv, "phi_storage": phs, "phase_field_integrator": "rk3" if rk3 else "euler",
            "mlups": mlups, "ms_per_step": ms,
            "bytes_per_lup": blup, "achieved_gbs": achieved, "frac": achieved / HBM_PEAK_GBS,
            "phase_volume_drift": abs(r1[0] - r0[0]) / r0[0], "nonfinite": int(r1[9]), "max_u": r1[7],
        }
        print(f"# {key}: {ms:.3f} ms/step, {mlups:.0f} MLUPS, {achieved:.0f} GB/s ({achieved / HBM_PEAK_GBS:.1%})",
              file=sys.stderr, flush=True)
        if not args.no_cpu_baseline:  # the oracle runs on the host: skipped with it
            variants[key]["error_vs_oracle"] = error_vs_oracle(st, curv, phs, rk3)
            print(f"#   vs FP64 oracle (64^3, 50 steps): u {variants[key]['error_vs_oracle']['u_rel_l2']:.2e}",
                  file=sys.stderr, flush=True)
    primary = next(iter(variants))
    v = variants[primary]
    traffic = (traffic_for(name, v["storage"])
               if (v["curvature"], v["phi_storage"], v["phase_field_integrator"]) == ("fd", "f64", "euler") else None)
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
                   "density_ratio": 10, "sigma": 0.005, "tau": tau, "storage": v["storage"],
                   "curvature": v["curvature"], "phi_storage": v["phi_storage"], "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": v["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": v["frac"], "traffic": traffic},
        "variants": variants,
        "copy_gbs": copy_gbs(),
        "kernel_sha": kernel_sha(),
    }
    if not args.no_batch:
        line["batch"] = batch_leg(min(args.steps, 50), min(args.warmup, 10), args.repeats)
        bt = line["batch"]
        print(f"# batch: {bt['mlups_batched']:.0f} MLUPS batched vs {bt['mlups_per_instance']:.0f} per instance "
              f"({bt['speedup']:.2f}x), tile {bt['tile']}, z-chunk {bt['zchunk']}", file=sys.stderr, flush=True)
    if not args.no_small_bubbles:
        line["small_bubbles"] = small_bubble_leg(min(args.steps, 50), min(args.warmup, 10), args.repeats,
                                                 args.size)
    if not args.no_cpu_baseline:
        print("# oracle on the host cores (cpu_baseline) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(shape, phi0, u0, params, nb, steps=args.cpu_steps)
        print(f"# cpu_baseline: {line['cpu_baseline']['value']:.2f} MLUPS ({line['cpu_baseline']['sample']})",
              file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
