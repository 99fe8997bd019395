"""FP64 CPU oracle of the accLB lattice update (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package.  The GPU product path never does.
"""
from .oracle import *  # noqa: F401,F403
