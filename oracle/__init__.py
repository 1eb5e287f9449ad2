"""FP64 CPU oracle for A-MMMSE / WMMSE precoding (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it and shares no code with it.
"""
from .ammse_oracle import *  # noqa: F401,F403
