"""Seeded synthetic inputs for the lattice update (initial fields and forcing tables).

This module builds initial conditions and forcing tables only; it holds none of
the time-stepping arithmetic.  The same arrays feed the FP64 oracle and the GPU
library, so both start from identical bits.

Layouts (all numpy, C order, x fastest):
  phi0   float64 [nz, ny, nx]        order parameter, 1 = liquid phase
  u0     float64 [3, nz, ny, nx]     SoA velocity (component major)
  pstar0 float64 [nz, ny, nx]        dimensionless pressure p* = p / (rho c_s^2)
  modes  float64 [M, 9]              forcing table, row = (kx, ky, kz, Re Ax, Im Ax,
                                     Re Ay, Im Ay, Re Az, Im Az); the body
                                     acceleration is a(x) = sum_m Re(A_m e^{i theta_m}),
                                     theta_m = 2 pi (kx x/nx + ky y/ny + kz z/nz).

Recipes follow the paper's workloads (Sec. 4 benchmarks, Sec. 5.1 HIT with a
large-scale time-independent forcing, Sec. 5.2 bubble-laden HIT) at the sizes the
tests and the benchmark use.  The equilibrium interface profile used for phi0 is
the tanh profile of Sec. 2.1.1 read with the Euclidean signed distance and
argument 2d/delta (the exact steady solution of Eq. (3) for kappa = 4D/delta).
"""
from __future__ import annotations

import math
import os

import numpy as np

__all__ = [
    "grid",
    "tanh_profile",
    "droplet",
    "bubble_pack",
    "planar_interface",
    "tgv",
    "solenoidal_field",
    "forcing_modes",
    "abc_modes",
    "abc_field",
    "random_u",
]


def grid(shape):
    """Integer lattice coordinates (z, y, x) broadcastable arrays for shape (nz, ny, nx)."""
    nz, ny, nx = shape
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    return z, y, x


def _wrap(d, n):
    """Periodic minimum-image displacement."""
    return d - n * np.round(d / n)


def tanh_profile(signed_dist, width):
    """phi = 1/2 (1 + tanh(2 d / delta)), d > 0 inside the phi = 1 phase."""
    return 0.5 * (1.0 + np.tanh(2.0 * signed_dist / width))


def droplet(shape, radius, width=4.0, center=None, seed=None, inside=1.0):
    """One sphere of the phi = `inside` phase (1 = droplet, 0 = bubble) in a periodic box.

    The centre is the box centre plus a seeded sub-cell offset U[-1/2, 1/2)^3
    when `seed` is given (or `center` when given explicitly, ordered (x, y, z)).
    Returns (phi0, center_xyz).
    """
    nz, ny, nx = shape
    if center is None:
        c = np.array([nx / 2.0, ny / 2.0, nz / 2.0])
        if seed is not None:
            c = c + np.random.default_rng(seed).uniform(-0.5, 0.5, size=3)
    else:
        c = np.asarray(center, dtype=np.float64)
    z, y, x = grid(shape)
    r = np.sqrt(_wrap(x - c[0], nx) ** 2 + _wrap(y - c[1], ny) ** 2 + _wrap(z - c[2], nz) ** 2)
    phi = tanh_profile(radius - r, width)
    if inside == 0.0:
        phi = 1.0 - phi
    return np.ascontiguousarray(phi), c


def planar_interface(shape, x0, width=4.0, axis=2):
    """Slab of phi = 1 between two planar interfaces (periodic), normal along `axis`
    (0 = z, 1 = y, 2 = x).  The slab is centred at x0 with half thickness n/4."""
    n = shape[axis]
    coords = np.arange(n, dtype=np.float64)
    d = n / 4.0 - np.abs(_wrap(coords - x0, n))
    prof = tanh_profile(d, width)
    sh = [1, 1, 1]
    sh[axis] = n
    return np.ascontiguousarray(np.broadcast_to(prof.reshape(sh), shape).copy())


def bubble_pack(shape, n_bubbles, diameter, width=4.0, seed=0, min_gap=None, max_tries=200000):
    """Seeded non-overlapping bubbles (phi = 0 inside) in a periodic box.

    `diameter` is a number or a (lo, hi) range sampled uniformly per bubble.
    Bubbles keep a periodic minimum-image clearance of (d_a + d_b)/2 + gap with
    gap = `width` by default.  phi0 = min_b 1/2 (1 + tanh(2 (|x - c_b| - R_b)/delta)).
    The profile is evaluated inside a box of half size R_b + 10 delta around
    each centre; beyond it tanh(2 d/delta) is 1 to double precision.
    Returns (phi0, centers [n,3] (x,y,z), radii [n]).
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    L = np.array([nx, ny, nz], dtype=np.float64)
    if np.isscalar(diameter):
        diam = np.full(n_bubbles, float(diameter))
    else:
        diam = rng.uniform(diameter[0], diameter[1], size=n_bubbles)
    gap = width if min_gap is None else min_gap
    centers = np.zeros((0, 3))
    radii = np.zeros(0)
    tries = 0
    for b in range(n_bubbles):
        r = diam[b] / 2.0
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("bubble_pack: could not place bubbles without overlap")
            c = rng.uniform(0.0, 1.0, size=3) * L
            if len(centers):
                d = _wrap(centers - c, L)
                dist = np.sqrt((d * d).sum(axis=1))
                if np.any(dist < radii + r + gap):
                    continue
            centers = np.vstack([centers, c])
            radii = np.append(radii, r)
            break
    # signed distance to the nearest bubble surface (positive outside = liquid)
    sd = np.full(shape, np.inf)
    for c, r in zip(centers, radii):
        h = int(math.ceil(r + 10.0 * width))
        axes = []
        for a, n in enumerate((nx, ny, nz)):
            if 2 * h + 2 >= n:
                idx = np.arange(n)
                disp = _wrap(idx - c[a], n)
            else:
                lo = int(math.floor(c[a])) - h
                raw = np.arange(lo, lo + 2 * h + 2)
                idx = raw % n
                disp = raw - c[a]
            axes.append((idx, disp))
        (ix, dx), (iy, dy), (iz, dz) = axes
        dist = np.sqrt(dx[None, None, :] ** 2 + dy[None, :, None] ** 2 + dz[:, None, None] ** 2) - r
        sel = np.ix_(iz, iy, ix)
        sd[sel] = np.minimum(sd[sel], dist)
    phi = np.where(np.isfinite(sd), tanh_profile(sd, width), 1.0)
    return np.ascontiguousarray(phi), centers, radii


def tgv(shape, u0=0.02, p0=1.0):
    """2-D Taylor-Green vortex in a 3-D periodic box, k = 2 pi / nx (nx == ny).

    u = u0 sin(kx) cos(ky), v = -u0 cos(kx) sin(ky), w = 0,
    p* = p0 - (3 u0^2 / 4)(cos 2kx + cos 2ky)   (rho0 = 1, c_s^2 = 1/3).
    Returns (u0 [3,nz,ny,nx], pstar0 [nz,ny,nx], k).
    """
    nz, ny, nx = shape
    k = 2.0 * math.pi / nx
    ky = 2.0 * math.pi / ny
    z, y, x = grid(shape)
    u = np.zeros((3,) + tuple(shape))
    u[0] = u0 * np.sin(k * x) * np.cos(ky * y) + 0.0 * z
    u[1] = -u0 * np.cos(k * x) * np.sin(ky * y) + 0.0 * z
    p = p0 - 0.75 * u0 * u0 * (np.cos(2 * k * x) + np.cos(2 * ky * y)) + 0.0 * z
    return np.ascontiguousarray(u), np.ascontiguousarray(p), k


def solenoidal_field(shape, rms=0.02, k0=4.0, seed=0):
    """Seeded random divergence-free (spectrally) velocity field.

    Spectrum E(k) ~ k^4 exp(-2 (k/k0)^2) (k in units of 2 pi / L), random
    complex Gaussian coefficients projected onto the plane normal to k, scaled so
    that sqrt(<|u|^2>/3) = rms.  Returns u [3,nz,ny,nx] float64.
    """
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    KZ = (np.fft.fftfreq(nz) * nz)[:, None, None]
    KY = (np.fft.fftfreq(ny) * ny)[None, :, None]
    KX = (np.fft.rfftfreq(nx) * nx)[None, None, :]
    K2 = KX * KX + KY * KY + KZ * KZ
    K = np.sqrt(K2)
    with np.errstate(divide="ignore", invalid="ignore"):
        amp = np.where(K > 0, np.sqrt(K ** 4 * np.exp(-2.0 * (K / k0) ** 2) / np.maximum(K2, 1.0)), 0.0)
    del K
    spec = []
    for _ in range(3):
        spec.append((rng.standard_normal(amp.shape) + 1j * rng.standard_normal(amp.shape)) * amp)
    del amp
    inv = np.where(K2 > 0, 1.0 / np.where(K2 > 0, K2, 1.0), 0.0)
    kdotv = (KX * spec[0] + KY * spec[1] + KZ * spec[2]) * inv
    spec[0] -= KX * kdotv
    spec[1] -= KY * kdotv
    spec[2] -= KZ * kdotv
    del kdotv, inv, K2
    try:
        import scipy.fft as sfft

        u = np.array([sfft.irfftn(spec[c], s=shape, axes=(0, 1, 2), workers=os.cpu_count()) for c in range(3)])
    except ImportError:
        u = np.array([np.fft.irfftn(spec[c], s=shape, axes=(0, 1, 2)) for c in range(3)])
    scale = rms / math.sqrt(float((u * u).sum(axis=0).mean()) / 3.0)
    u *= scale
    return np.ascontiguousarray(u)


def _shell_vectors(kmax2=4):
    """Integer wave vectors with 0 < |k|^2 <= kmax2 (32 of them for kmax2 = 4)."""
    out = []
    r = int(math.isqrt(kmax2))
    for kz in range(-r, r + 1):
        for ky in range(-r, r + 1):
            for kx in range(-r, r + 1):
                k2 = kx * kx + ky * ky + kz * kz
                if 0 < k2 <= kmax2:
                    out.append((kx, ky, kz))
    return out


def forcing_modes(amplitude=1e-5, seed=0, kmax2=4):
    """Large-scale forcing on the shells 0 < |k|^2 <= kmax2 with seeded random phases.

    Each Hermitian pair (k, -k) gets a random complex amplitude vector normal to k
    (solenoidal), the -k row holding the complex conjugate, so the field is real.
    Scaled so that the per-component rms of a(x) over the box is `amplitude`
    (Parseval: <|a|^2> = sum over the table of |A_m|^2).  Time independent, like
    the ABC forcing of Sec. 5.1.  Returns the [M, 9] table.
    """
    rng = np.random.default_rng(seed)
    ks = _shell_vectors(kmax2)
    rows = {}
    for k in ks:
        if k in rows:
            continue
        neg = (-k[0], -k[1], -k[2])
        kv = np.array(k, dtype=np.float64)
        v = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        v = v - kv * (kv @ v) / (kv @ kv)
        v = v * np.exp(2j * math.pi * rng.uniform())
        rows[k] = v
        rows[neg] = np.conj(v)
    table = np.zeros((len(ks), 9))
    for m, k in enumerate(ks):
        A = rows[k]
        table[m, 0:3] = k
        table[m, 3::2] = A.real
        table[m, 4::2] = A.imag
    power = float((table[:, 3:] ** 2).sum())
    table[:, 3:] *= amplitude / math.sqrt(power / 3.0)
    return table


def abc_modes(amplitude, kf=1):
    """The ABC forcing of Sec. 5.1, A (sin kz + cos ky, sin kx + cos kz, sin ky + cos kx)
    with k = 2 pi kf / L, written as a six-row mode table."""
    h = 0.5 * amplitude
    t = np.zeros((6, 9))
    # (kx,ky,kz), then (Ax, Ay, Az) complex
    spec = [
        ((kf, 0, 0), (0, -1j * h, h)),
        ((-kf, 0, 0), (0, 1j * h, h)),
        ((0, kf, 0), (h, 0, -1j * h)),
        ((0, -kf, 0), (h, 0, 1j * h)),
        ((0, 0, kf), (-1j * h, h, 0)),
        ((0, 0, -kf), (1j * h, h, 0)),
    ]
    for m, (k, A) in enumerate(spec):
        t[m, 0:3] = k
        A = np.asarray(A, dtype=np.complex128)
        t[m, 3::2] = A.real
        t[m, 4::2] = A.imag
    return t


def abc_field(shape, amplitude, kf=1):
    """ABC field evaluated on the grid (cubic box assumed for k = 2 pi kf / n).
    Returns [3, nz, ny, nx]."""
    nz, ny, nx = shape
    z, y, x = grid(shape)
    kx, ky, kz = 2 * math.pi * kf / nx, 2 * math.pi * kf / ny, 2 * math.pi * kf / nz
    f = np.zeros((3,) + tuple(shape))
    f[0] = amplitude * (np.sin(kz * z) + np.cos(ky * y)) + 0 * x
    f[1] = amplitude * (np.sin(kx * x) + np.cos(kz * z)) + 0 * y
    f[2] = amplitude * (np.sin(ky * y) + np.cos(kx * x)) + 0 * z
    return np.ascontiguousarray(f)


def random_u(shape, scale=0.01, seed=0):
    """Smooth-free white-noise velocity (for conservation and parity probes)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(-scale, scale, size=(3,) + tuple(shape)))


def bubble_box_ensemble(count=128, seed=0, edges=(32, 96), n_range=(1, 8), d_range=(6.0, 20.0),
                        ratio_range=(1.0, 10.0), width=4.0):
    """Seeded ensemble of independent bubble-in-box instances of uneven size.

    Instance k: a cubic periodic box with edge drawn from the multiples of 8 in
    `edges`, n_k bubbles (uniform in `n_range`) with diameters uniform in
    `d_range`, and a density ratio uniform in `ratio_range`.  Where the bubbles
    do not fit without overlap, the count is lowered until they do.  Returns a
    list of dicts with keys shape, phi0, ratio, n_bubbles.
    """
    rng = np.random.default_rng(seed)
    choices = np.arange(edges[0], edges[1] + 1, 8)
    out = []
    for k in range(count):
        n = int(choices[rng.integers(0, len(choices))])
        nb = int(rng.integers(n_range[0], n_range[1] + 1))
        ratio = float(rng.uniform(*ratio_range))
        sub = int(rng.integers(0, 2 ** 31))
        while True:
            try:
                phi0, _, _ = bubble_pack((n, n, n), nb, d_range, width=width, seed=sub, max_tries=20000)
                break
            except RuntimeError:
                nb -= 1
                if nb == 0:
                    raise
        out.append({"shape": (n, n, n), "phi0": phi0, "ratio": ratio, "n_bubbles": nb})
    return out
