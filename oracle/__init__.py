"""CPU FP64 oracle for one HOT implicit MPM step (test infrastructure only).

This package is the independent reference that the HIP path is checked
against.  It is plain numpy/scipy written from the paper (Hierarchical
Optimization Time Integration for CFL-rate MPM Stepping): slow, unblocked and
unfused.  It shares no code with the GPU library.  Only ``tests/``, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may
import it; the product path never does.
"""
from .hot_oracle import *  # noqa: F401,F403
