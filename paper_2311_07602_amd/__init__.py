"""lrbg: batched low-rank GEMM for AMD Instinct MI355X (gfx950).

The compute path is the C-ABI library ``liblrbg.so`` (hand-written HIP
kernels) declared in ``include/lrbg.h``; :mod:`.lrbg` is a thin ctypes binding
with the same entry-point names.  :mod:`.inputs` holds the seeded synthetic
input generators; :mod:`.serve` the continuous-batching request loop.

Importing the package loads nothing native; the library is loaded on first
use and raises if it has not been built.
"""
__version__ = "0.1.0"
