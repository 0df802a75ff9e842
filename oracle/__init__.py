"""CPU oracle for compressed matrix multiplication in the FWHT form.

TEST INFRASTRUCTURE ONLY.  Plain float64 NumPy written from the paper
(Andersson & Karppa, "Engineering Compressed Matrix Multiplication with the
Fast Walsh-Hadamard Transform"): Algorithm 1, the XOR-convolution identity of
Section 2 / Section 3.2, the multiply-add-shift hash of Section 4.2 and the
two other families it names, Pagh's FFT form (Section 3.1), and the
correctness counters and per-repetition estimates of the evaluation
(Sections 5.3 and 5.4).
Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import it.  It shares no code with the HIP library and the
library never calls it.

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
brute force, library routines and hand-worked examples; none is marked
"parity unpinned".
"""
from .cmm_oracle import *  # noqa: F401,F403
