"""Reference oracle for batched low-rank products (test infrastructure only).

Only ``tests/``, the smoke check and the CPU-baseline leg of ``bench.py``
may import this package.  The GPU library never does.
"""
from .oracle import *  # noqa: F401,F403
