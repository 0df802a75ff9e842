"""CPU oracle for compressed matrix multiplication in the FWHT form.

TEST INFRASTRUCTURE ONLY.  Plain float64 NumPy written from the paper
(Andersson & Karppa, "Engineering Compressed Matrix Multiplication with the
Fast Walsh-Hadamard Transform"): Algorithm 1, the XOR-convolution identity of
Section 2 / Section 3.2, and the multiply-add-shift hash of Section 4.2.
Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import it.  It shares no code with the HIP library and the
library never calls it.

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
brute force, library routines and hand-worked examples; none is marked
"parity unpinned".
"""
from .cmm_oracle import *  # noqa: F401,F403
