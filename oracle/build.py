"""Compile the C oracle into oracle/liboracle.so with gcc (OpenMP, no FMA contraction).

TEST INFRASTRUCTURE: the product never loads the result.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False, src=None, out=None, warnings=True):
    """Compile oracle.c (or `src`, a copy of it, with -I pointing at this
    directory for oracle.h) into liboracle.so (or `out`)."""
    src = src or os.path.join(HERE, "oracle.c")
    out = out or LIB
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall" if warnings else "-w", "-I", HERE, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build_planted(replacements, workdir):
    """A copy of the oracle with mistakes planted in its source, for tests that
    show a pin catches them: each (old, new) pair must occur exactly once in
    oracle.c.  Returns the path of the compiled copy under `workdir`."""
    with open(os.path.join(HERE, "oracle.c")) as f:
        text = f.read()
    for old, new in replacements:
        n = text.count(old)
        if n != 1:
            raise ValueError(f"planted mistake: {old!r} occurs {n} times in oracle.c")
        text = text.replace(old, new)
    src = os.path.join(workdir, "oracle_planted.c")
    with open(src, "w") as f:
        f.write(text)
    # a planted mistake may leave a variable unused: no warnings for the copy
    return build(src=src, out=os.path.join(workdir, "liboracle_planted.so"), warnings=False)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
