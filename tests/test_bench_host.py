"""Host logic of bench.py that needs no GPU: variant names, algorithmic bytes
per lattice update, and the refusal of more than one GPU."""
import os
import subprocess
import sys

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
