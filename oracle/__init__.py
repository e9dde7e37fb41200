"""FP64 CPU oracle of the Gaussian-splatting mapping step (test infrastructure).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It shares no code with the HIP implementation.
"""
from .oracle import *  # noqa: F401,F403
