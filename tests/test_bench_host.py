"""Host logic of bench.py that needs no GPU: variant names, algorithmic bytes
per lattice update, the refusal of more than one GPU, the shared bubble
recipe and the shipped network weights."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_variant_names():
    assert bench.parse_variant("f32") == ("f32", "fd", "f64", False)
    assert bench.parse_variant("f16:mlp") == ("f16", "mlp", "f64", False)
    assert bench.parse_variant("f16:fix32") == ("f16", "fd", "fix32", False)
    assert bench.parse_variant("f32:mlp:rk3") == ("f32", "mlp", "f64", True)
    with pytest.raises(SystemExit):
        bench.parse_variant("f32:bogus")


def test_algorithmic_bytes_per_update():
    # 27 population reads + 27 writes, phi read + write, u read + write
    assert bench.bytes_per_lup("f32") == 27 * 4 * 2 + 8 + 8 + 12 + 12 == 256
    assert bench.bytes_per_lup("f16") == bench.bytes_per_lup("bf16") == 148
    assert bench.bytes_per_lup("f32", "fix32") == 248
    assert bench.bytes_per_lup("f16", "fix32") == 140
    # two more phase-field stages of 36 bytes each
    assert bench.bytes_per_lup("f32", rk3=True) == 328
    assert bench.bytes_per_lup("f16", rk3=True) == 220


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bubble_recipe_is_shared_by_the_workload_and_the_small_bubble_report():
    """workload() and the Laplace report at rest draw the same seeded bubbles."""
    shape, phi0, centers, radii, nb = bench.bubbles(64, seed=0, diameter=(4.0, 6.0))
    shape2, phi0b, u0, params, nb2 = bench.workload(64, seed=0, diameter=(4.0, 6.0))
    assert shape == shape2 and nb == nb2 == 1
    np.testing.assert_array_equal(phi0, phi0b)
    assert np.all((radii >= 2.0) & (radii <= 3.0))
    assert {k: params[k] for k in bench.TWO_PHASE} == bench.TWO_PHASE and "modes" in params


def test_shipped_network_weights_have_the_network_shape():
    """The trained network the learned-curvature variants load: 6 212 finite
    fp16 values (27x64 + 64, 64x64 + 64, 4x64 + 4), not a placeholder."""
    w = np.load(bench.WEIGHTS, allow_pickle=False)
    assert w.dtype == np.float16 and w.shape == (6212,)
    assert np.all(np.isfinite(w)) and np.abs(w).max() > 0.1 and np.count_nonzero(w) > 6000
