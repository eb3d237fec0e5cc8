"""Serial FP64 CPU oracle of the per-level AMR hydro update (test infrastructure).

Only tests/, the smoke check in __graft_entry__ and the CPU-baseline leg of
bench.py may import this package.  The product path never does.
"""
from .oracle import *  # noqa: F401,F403
