"""The C-ABI library loads and exports every entry point include/lbm.h declares;
host-side validation runs without a GPU (no compute calls here)."""
import ctypes as C
import os
import re

import pytest

from paper_2505_01126_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = lbm.load_library()
    names = _declared()
    assert "lbm_init" in names and "lbm_step" in names and "lbm_moments" in names and "lbm_reduce" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(lbm.SYMBOLS)


def test_abi_version_and_constants():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    ver = int(re.search(r"#define LBM_ABI_VERSION (\d+)", text).group(1))
    assert lbm.lbm_abi_version() == ver
    assert int(re.search(r"#define LBM_NRED (\d+)", text).group(1)) == lbm.NRED
    assert int(re.search(r"#define LBM_MLP_NPARAM (\d+)", text).group(1)) == lbm.MLP_NPARAM
    assert C.sizeof(lbm.lbm_config) == 160


def test_config_struct_matches_header(tmp_path):
    """The ctypes mirror of lbm_config has the C compiler's size and offsets."""
    import shutil
    import subprocess

    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    fields = [f for f, _ in lbm.lbm_config._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lbm.h"\nint main(void) {\n'
                   '  printf("%zu\\n", sizeof(lbm_config));\n'
                   + "".join(f'  printf("%zu\\n", offsetof(lbm_config, {f}));\n' for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert out[0] == C.sizeof(lbm.lbm_config)
    assert out[1:] == [getattr(lbm.lbm_config, f).offset for f in fields]


def test_workspace_bytes_counts_state():
    cfg, _ = lbm.make_config((64, 64, 64), 0.8)
    one = lbm.lbm_workspace_bytes(cfg)
    N = 64 ** 3
    assert one >= 2 * 27 * 4 * N
    cfg2, _ = lbm.make_config((64, 64, 64), 0.8, two_phase=True, storage="f16")
    two = lbm.lbm_workspace_bytes(cfg2)
    assert two >= 2 * 27 * 2 * N + 2 * 8 * N + 2 * 12 * N
    assert two < 2 * 27 * 2 * N + 2 * 8 * N + 2 * 12 * N + (1 << 20)
    # int32 fixed-point phi: two 4-byte fields instead of two 8-byte ones
    cfg3, _ = lbm.make_config((64, 64, 64), 0.8, two_phase=True, storage="f16", phi_storage="fix32")
    assert lbm.lbm_workspace_bytes(cfg3) == two - 2 * 4 * N


@pytest.mark.parametrize("kw", [dict(tau=0.5), dict(tau=0.8, shape=(4, 64, 64)),
                                dict(tau=0.8, shape=(8, 4097, 4097)),
                                dict(tau=0.8, storage="f16", modes=[[3, 0, 0] + [0] * 6]),
                                dict(tau=0.8, two_phase=True, phi_storage=2),
                                dict(tau=0.8, two_phase=True, tau_g=0.45),
                                dict(tau=0.8, two_phase=True, gravity=(0.0, float("nan"), 0.0)),
                                dict(tau=0.8, two_phase=True, ac_rk3=1, phi_storage="fix32")])
def test_invalid_configs_rejected_on_host(kw):
    shape = kw.pop("shape", (16, 16, 16))
    tau = kw.pop("tau")
    cfg, keep = lbm.make_config(shape, tau, **kw)
    assert lbm.lbm_workspace_bytes(cfg) == 0
    h = C.c_void_p()
    rc = lbm.load_library().lbm_init(C.byref(h), C.byref(cfg), None, 0, None, None, None, None)
    assert rc == lbm.LBM_EINVAL
    assert lbm.load_library().lbm_last_error(None).decode()


def test_strerror_texts():
    L = lbm.load_library()
    for code in (0, -1, -2, -3, -4):
        assert L.lbm_strerror(code).decode()
