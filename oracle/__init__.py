"""FP64 reference (oracle) for the accelerated shiftable bilateral filter.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The GPU library never imports,
links or calls anything here, and nothing here uses the GPU library.
"""
from .oracle import *  # noqa: F401,F403
