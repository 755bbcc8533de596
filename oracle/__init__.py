"""HAMLET oracle: a plain, slow FP64 CPU reference of the reconstruction.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the CPU-baseline leg of the benchmark may import anything from here.  It
shares no code with the GPU library and imports nothing from it.
"""
from . import fft, model, philox, hmc  # noqa: F401
