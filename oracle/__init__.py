"""CPU oracle for DET-LSH: test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package. The GPU library never does, and the two share no code.
"""
from .detlsh import *  # noqa: F401,F403
