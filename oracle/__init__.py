"""FP64 CPU oracle (test infrastructure only).

A plain, slow, NumPy complex128 implementation of the IRLS structured
low-rank recovery of arXiv 1704.04511, written from the paper.  Only the test
suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the HIP library never does, and the two share no
code.  Pins against closed forms, brute force and textbook routines live in
``tests/test_oracle_*.py``.
"""
from .slr import *  # noqa: F401,F403
from .slr import __all__  # noqa: F401
