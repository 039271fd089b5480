"""FP64 CPU oracle (test infrastructure).

Only tests/, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library; see oracle.c for the routines and their sources in the paper.
"""
from .oracle import *  # noqa: F401,F403
