"""Compile the HIP sources of the package into paper_2505_01126_amd/liblbm.so (gfx950)."""
import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "liblbm.so")
SOURCES = ["lbm_step_s0.hip", "lbm_step_s1.hip", "lbm_step_s2.hip", "lbm_kernels.hip", "lbm_mlp.hip", "lbm_api.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off on this target (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose=False, extra=None):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    # one object per source, compiled concurrently, then one link
    with tempfile.TemporaryDirectory() as d:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(d, src.replace(".hip", ".o"))
            cmd = [hipcc] + [f for f in HIPCC_FLAGS if f != "-shared"] + list(extra or []) + inc + [
                "-c", "-o", obj, os.path.join(PKG, "csrc", src)]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd)))
            objs.append(obj)
        failed = [cmd for cmd, p in procs if p.wait() != 0]
        if failed:
            raise subprocess.CalledProcessError(1, failed[0])
        link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
