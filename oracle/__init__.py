"""FP64 CPU oracle for the Lyman-alpha pair sums (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library.
"""
from .lya_oracle import *  # noqa: F401,F403
