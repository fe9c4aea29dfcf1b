"""FP64 CPU oracle (test infrastructure only).

Only the test suite, the entry point's smoke check and the benchmark's CPU
baseline leg may import this package.  The GPU library never does.
"""
from .propagator import *  # noqa: F401,F403
