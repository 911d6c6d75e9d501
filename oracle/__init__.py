"""FP64 CPU oracle (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library never does.  See oracle.py.
"""
from .oracle import *  # noqa: F401,F403
