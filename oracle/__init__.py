"""Oracle package: plain FP64 CPU reference implementations.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.
"""
from . import rgmres  # noqa: F401
