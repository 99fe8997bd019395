"""Batches of independent boxes in one persistent launch per step.

A box advanced inside a batch must give bit-identical fields to the same box
advanced alone: the work items run the same tile code, and no result depends
on the z-chunk length or on which workgroup takes an item.  Covered: uneven
and ragged box shapes, different physical parameters per box, odd and even
step counts (graph replays of step pairs plus single launches), FD and learned
curvature, members stepped on their own between batch steps, the autotuner,
cached and non-temporal output stores, and rejected mixes.  One member is also checked against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle as O
from parity import check
from paper_2505_01126_amd import inputs as I

pytestmark = pytest.mark.gpu

# the last box's rows fill whole 128-byte lines (nx = 128): alone (tile 64) its
# outputs are stored with the non-temporal policy, in a batch with 16-bit
# storage and tile 32 with the default one; the fields must not differ
SHAPES = [(16, 20, 70), (32, 32, 32), (40, 24, 48), (20, 36, 20), (24, 8, 96), (16, 12, 128)]


def _boxes(storage, curv, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for k, shape in enumerate(SHAPES):
        nz, ny, nx = shape
        r = float(rng.uniform(3.0, 5.0))
        center = (rng.uniform(r + 2, nx - r - 2), rng.uniform(0, ny), rng.uniform(0, nz))
        phi0, _ = I.droplet(shape, r, 4.0, center=center, inside=1.0 if k % 2 == 0 else 0.0)
        u0 = I.random_u(shape, 0.01, seed=seed + 10 + k)
        kw = dict(tau=float(rng.uniform(0.6, 1.0)), rho_l=1.0, rho_g=float(1.0 / rng.uniform(1.0, 10.0)),
                  sigma=float(rng.uniform(0.005, 0.02)), mobility=0.05, width=4.0, p0=0.0, storage=storage,
                  curv_mode=curv)
        out.append((shape, phi0, u0, kw))
    return out


def _make(boxes, w16=None):
    from paper_2505_01126_amd import lbm

    gs = []
    for shape, phi0, u0, kw in boxes:
        kw = dict(kw)
        tau = kw.pop("tau")
        g = lbm.Lattice(shape, tau, phi0=phi0, u0=u0, **kw)
        if w16 is not None:
            g.set_mlp(w16)
        gs.append(g)
    return gs


def _fields(g):
    return {k: v.clone() for k, v in g.moments().items()}


def _weights():
    import torch

    w = np.random.default_rng(3).standard_normal(6212) * 0.25
    w[-3:] = [0.6, 0.5, 0.4]
    return torch.tensor(w.astype(np.float16).view(np.int16), device="cuda")


def _assert_same(a, b, what):
    import torch

    for k in a:
        assert torch.equal(a[k], b[k]), f"{what}: field {k} differs"


@pytest.mark.parametrize("storage,curv,tiling", [("f16", "fd", None), ("f16", "mlp", None), ("f32", "fd", None),
                                                 ("f16", "fd", (32, 8)), ("f16", "mlp", (32, 16)),
                                                 ("f32", "fd", (32, 64))])
def test_batch_bit_identical_to_single_boxes(storage, curv, tiling):
    from paper_2505_01126_amd import lbm

    boxes = _boxes(storage, curv)
    w16 = _weights() if curv == "mlp" else None
    alone = _make(boxes, w16)
    for g in alone:
        g.step(7)
    ref = [_fields(g) for g in alone]
    members = _make(boxes, w16)
    b = lbm.Batch(members)
    if tiling is not None:
        b.set_tiling(*tiling)  # 32 x 8 tiles: two x-rows per wave
    b.step(3)  # one graph replay (2 steps) + one single launch
    b.step(4)  # realign launch, one replay, tail launch
    for i, g in enumerate(members):
        assert g.steps == 7
        _assert_same(_fields(g), ref[i], f"box {i} {SHAPES[i]}")
    b.close()


def test_batch_member_stepped_alone_and_tuned():
    from paper_2505_01126_amd import lbm

    boxes = _boxes("f16", "fd", seed=1)
    alone = _make(boxes)
    members = _make(boxes)
    b = lbm.Batch(members)
    b.step(2)
    members[1].step(1)  # on its own: the batch must pick up the new state
    b.step(2)
    tile, zc = b.tune(2)  # 8 candidates x (1 + 2) steps, every tile width and z-chunk
    assert tile in (64, 32) and zc in (8, 16, 32, 64)
    assert b.tune(2) == (tile, zc)  # cached: no further steps
    b.step(3)
    total = [2 + 2 + 24 + 3] * len(boxes)
    total[1] += 1
    for i, g in enumerate(members):
        assert g.steps == total[i]
        alone[i].step(total[i])
        _assert_same(_fields(g), _fields(alone[i]), f"box {i}")
    print(f"autotuned tile {tile}, z-chunk {zc}")
    b.close()


def test_batch_member_matches_oracle():
    from paper_2505_01126_amd import lbm

    boxes = _boxes("f32", "fd", seed=2)
    members = _make(boxes)
    b = lbm.Batch(members)
    b.step(10)
    shape, phi0, u0, kw = boxes[2]
    kw = {k: v for k, v in kw.items() if k not in ("storage", "curv_mode")}
    tau = kw.pop("tau")
    o = O.Oracle(shape, tau, phi0=phi0, u0=u0, **kw)
    o.step(10)
    mo = o.moments()
    m = {k: v.double().cpu().numpy() for k, v in members[2].moments().items()}
    check(m, mo, "f32", "batch member vs oracle", phi_bar=1e-5, drho=1.0)
    b.close()


def test_batch_rejects_mixed_members():
    from paper_2505_01126_amd import lbm

    a = _make(_boxes("f16", "fd")[:1])[0]
    c = _make(_boxes("f32", "fd")[:1])[0]
    with pytest.raises(lbm.LbmError):
        lbm.Batch([a, c])
    with pytest.raises(lbm.LbmError):
        lbm.Batch([a, a])
    with pytest.raises(lbm.LbmError):
        lbm.Batch([])
    b = lbm.Batch([a])
    with pytest.raises(lbm.LbmError):
        b.set_tiling(48, 8)
    b.close()
