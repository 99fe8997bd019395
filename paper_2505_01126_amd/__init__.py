"""MI355X lattice update of accLB (arXiv 2505.01126): regularised D3Q27 LB with
phase-field forcing, coupled to a conservative Allen-Cahn field.

The compute path is liblbm.so (HIP, gfx950) behind the C ABI in include/lbm.h;
`lbm` is its ctypes binding and `inputs` builds seeded initial conditions.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "lbm"]
