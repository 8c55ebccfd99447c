"""CPU oracle -- test infrastructure only.

Plain, untiled, loop-by-loop FP64 C implementations of the stencil proxies
(built with gcc -O2 -ffp-contract=off -fopenmp, no fast-math), wrapped with
ctypes.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
use this package; the HIP product path never imports it, and this package
imports nothing from the product package.
"""
from .build import build, load  # noqa: F401
