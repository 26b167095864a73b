"""FP64 CPU oracle for the GAP regression hot path -- test infrastructure only.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  It shares no code with the GPU library and never imports it.
"""
from .gap_oracle import *  # noqa: F401,F403
