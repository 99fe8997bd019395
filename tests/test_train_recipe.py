"""Host-side pieces of the learned-curvature training recipe (no GPU).

The network itself is trained by the library's kernels (test_gpu_mlp.py,
test_learned_curvature_gain.py); these pin the row transforms around it:
the 48 cube symmetries applied to a training row, the |grad phi|^2 weight of
a row, the radius law and the Laplace-consistent label's profile integral.
"""
import math

import numpy as np
import pytest
import torch

from paper_2505_01126_amd import inputs as I
from paper_2505_01126_amd import train_curvature as tc

OFFS = np.array([(i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1) for i in range(27)], dtype=np.float64)


def test_cube_symmetries_form_the_group_of_48():
    cols, ycols, ysign = tc.cube_symmetries()
    assert cols.shape == (48, 32) and ycols.shape == (48, 4) and ysign.shape == (48, 4)
    # each is a permutation of the 27 stencil columns that leaves the padding and the centre in place
    for c in cols:
        assert sorted(c.tolist()) == list(range(32))
        assert (c[27:] == np.arange(27, 32)).all() and c[13] == 13
    # 48 distinct maps, closed under composition
    keys = {tuple(c) for c in cols}
    assert len(keys) == 48
    for a in cols[::5]:
        for b in cols[::7]:
            assert tuple(a[b]) in keys
    # K is never moved or flipped
    assert (ycols[:, 0] == 0).all() and (ysign[:, 0] == 1.0).all()


def test_cube_symmetry_turns_stencil_and_normal_together():
    """A linear field phi = n . x has the stencil n . o_i; after a symmetry the
    stencil must be that of the transformed normal (a wrong sign or a
    transposed permutation fails here)."""
    cols, ycols, ysign = tc.cube_symmetries()
    rng = np.random.default_rng(0)
    for t in range(48):
        n = rng.standard_normal(3)
        x = np.zeros(32)
        x[:27] = OFFS @ n
        y = np.concatenate([[0.5], n])
        yt = y[ycols[t]] * ysign[t]
        np.testing.assert_allclose(x[cols[t]][:27], OFFS @ yt[1:], atol=1e-14)
        assert yt[0] == 0.5


def test_cube_symmetry_of_a_sphere_stencil():
    """The stencil of a sphere seen from a cell turns into the stencil seen from
    the mirrored / permuted cell position, with the radial normal turned alike."""
    cols, ycols, ysign = tc.cube_symmetries()
    R, c = 5.0, np.array([0.3, -0.2, 0.1])
    cell = np.array([4.0, 2.0, -1.0])
    phi = lambda p: 0.5 * (1.0 + np.tanh(2.0 * (R - np.linalg.norm(p - c, axis=-1)) / 4.0))  # noqa: E731
    for t in (1, 7, 20, 47):
        perm = [ycols[t][1 + a] - 1 for a in range(3)]
        sg = ysign[t][1:]
        T = np.zeros((3, 3))
        for a in range(3):
            T[a, perm[a]] = sg[a]
        x = np.zeros(32)
        x[:27] = 2.0 * phi(cell + OFFS) - 1.0
        # the same sphere turned by T, seen from the turned cell
        phi_t = lambda p: 0.5 * (1.0 + np.tanh(2.0 * (R - np.linalg.norm(p - T @ c, axis=-1)) / 4.0))  # noqa: E731
        xt = np.zeros(32)
        xt[:27] = 2.0 * phi_t(T @ cell + OFFS) - 1.0
        np.testing.assert_allclose(x[cols[t]], xt, atol=1e-13)
        nrm = (c - cell) / np.linalg.norm(c - cell)  # toward phi = 1
        y = np.concatenate([[0.4], nrm])
        np.testing.assert_allclose((y[ycols[t]] * ysign[t])[1:], T @ nrm, atol=1e-14)


def test_stencil_grad2_is_the_lattice_gradient_of_the_fp16_inputs():
    rng = np.random.default_rng(1)
    rows = []
    want = []
    for _ in range(20):
        phi = rng.uniform(0.0, 1.0, 27)
        x = np.zeros(32, dtype=np.float16)
        x[:27] = (2.0 * phi - 1.0).astype(np.float16)
        rows.append(x.view(np.int16))
        xv = x[:27].astype(np.float64)
        w = np.array([np.prod([(2.0 / 3.0 if o == 0 else 1.0 / 6.0) for o in off]) for off in OFFS])
        g = 3.0 * (w[:, None] * OFFS * ((xv + 1.0) / 2.0)[:, None]).sum(0)
        want.append((g * g).sum())
    got = tc.stencil_grad2(torch.tensor(np.array(rows))).double().numpy()
    np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-9)
    # the centre value does not enter a gradient; a constant stencil has none
    const = np.zeros(32, dtype=np.float16)
    const[:27] = 0.25
    assert float(tc.stencil_grad2(torch.tensor(const.view(np.int16)[None, :]))) < 1e-12


def test_inverse_radius_law_spreads_interface_cells_over_radii():
    rng = np.random.default_rng(2)
    radii = np.concatenate([tc._place(rng, 400, 4, 2.0, 10.0, 4.0, "inverse")[1] for _ in range(400)])
    assert radii.min() >= 2.0 and radii.max() <= 10.0
    # 1/R is uniform: each of four equal 1/R bins holds a quarter of the radii
    h, _ = np.histogram(1.0 / radii, bins=4, range=(0.1, 0.5))
    assert np.all(np.abs(h / len(radii) - 0.25) < 0.04)
    # so the interface area (R^2) per unit of radius is about even: [2, 4) holds
    # half the area of [6, 10] (a uniform radius law gives 0.07)
    a_small = (radii[radii < 4.0] ** 2).sum()
    a_large = (radii[radii >= 6.0] ** 2).sum()
    assert 0.35 < a_small / a_large < 0.7
    with pytest.raises(ValueError):
        tc._place(rng, 40, 1, 2.0, 10.0, 4.0, "log")


def test_csf_integral_approaches_the_planar_value_as_the_sphere_grows():
    """I = (3 delta / 2) int |grad phi|^2 dr is 1 for the continuous planar tanh
    profile of width delta (the normalisation of the surface-tension force).
    With the lattice gradient of a plane, which is the central difference
    across it, the planar value is a 1-D sum; the sphere's I, a 3-D sum over
    the sphere's cells divided by 4 pi r^2, must approach it as R grows and
    fall below it on a small sphere."""
    # continuous planar value, by quadrature: (3 delta/2) int (1/delta^2) sech^4(2 s/delta) ds = 1
    s = np.linspace(-40, 40, 200001)
    dphi = (1.0 / 4.0) / np.cosh(2.0 * s / 4.0) ** 2
    assert abs(1.5 * 4.0 * np.trapezoid(dphi ** 2, s) - 1.0) < 1e-9
    # the lattice's planar value, averaged over the plane's offset from the grid
    planar = []
    for off in np.linspace(0.0, 1.0, 8, endpoint=False):
        xs = np.arange(-60, 61) + off
        ph = I.tanh_profile(xs, 4.0)
        g = 0.5 * (ph[2:] - ph[:-2])
        planar.append(1.5 * 4.0 * float((g * g).sum()))
    planar = float(np.mean(planar))
    assert 0.9 < planar < 0.97  # the central difference flattens the tanh's slope
    n = 64
    vals = {}
    for R in (4.0, 20.0):
        c = np.array([31.6, 32.3, 31.9])
        z, y, x = I.grid((n, n, n))
        d = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
        vals[R] = tc.csf_integral(I.tanh_profile(R - d, 4.0), np.array([c]))[0]
    assert abs(vals[20.0] / planar - 1.0) < 0.01
    assert vals[4.0] < vals[20.0] - 0.02 and math.isfinite(vals[4.0])
