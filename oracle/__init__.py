"""CPU oracle for the balanced-tree FMM evaluation pass (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
use this package.  It wraps `liboracle.so` (plain C, binary64, built by
`oracle/build.sh`) with ctypes and shares no code with the GPU library.
"""
from .oracle import *  # noqa: F401,F403
