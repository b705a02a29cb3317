"""CPU FP64 reference of the Noise2Fast loop.

Test infrastructure only: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are its only callers.  The product never imports it.
"""
from . import n2f_oracle  # noqa: F401
