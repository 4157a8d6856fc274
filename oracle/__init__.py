"""Plain FP64 CPU oracle for the checkerboard SU(3) heat-bath sweep.

TEST INFRASTRUCTURE ONLY: loaded by the test suite, the package smoke test and
the CPU-baseline leg of the benchmark, never by the GPU product path.
"""
from .su3ref import Oracle, lib, load  # noqa: F401
