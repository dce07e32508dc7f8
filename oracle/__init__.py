"""FP64 CPU oracle for the hybrid BEM/BIEM diffusion-curve method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute this package: only the test suite, the smoke check of the
package entry point and the CPU-baseline leg of the benchmark use it.  It
shares no code with the GPU library (which is written in C++/HIP); the two
meet only through the seeded input arrays of ``scenegen``.
"""
from .dcoracle import *  # noqa: F401,F403
from . import adaptive  # noqa: F401
