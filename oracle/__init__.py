"""FP64 CPU oracle for the EI-FP scheme -- test infrastructure, not product code.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  The GPU library neither imports nor links it.
"""
from .oracle import *  # noqa: F401,F403
