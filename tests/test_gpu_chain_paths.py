"""Collision fix-up paths of the fused compress that the other tests do not
reach: in the layout with a separate transpose buffer, repetitions whose
chains all have two rows and number more than one descriptor slot per
thread (512) in an operand, so that waves hold several live slots.  The
n = 8192 workload's keys give such repetitions once the transform windows
are chosen; float32 rows of 8192 elements still sit beside a transpose
buffer.  Sparse +-1 operands keep the float32 path exact, so p must equal
the oracle's bucket sums (Algorithm 1 Compress) bit for bit."""
import numpy as np
import pytest

import oracle as O
import paper_2601_09477_amd as cmm
from workloads import draw_keys
from tests.gpu_util import announce, dev, host, torch

pytestmark = pytest.mark.gpu

LB = 13          # log2 of the slice the fused kernel transforms (b_lo)
MAX_WINDOW = 5   # largest right rotation of the bucket bits considered


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch().cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()


def _chains(tab, log2b, s):
    """Rows per lo-bucket after rotating the bucket bits right by s: the
    number of two-row chains and of longer ones, and the window cost (rows
    beyond the first, plus 8 per row beyond the sixth)."""
    v = ((tab & ((1 << log2b) - 1)) >> s) & ((1 << LB) - 1)
    c = np.bincount(v, minlength=1 << LB)
    cost = int(np.sum(np.maximum(c - 1, 0))) + 8 * int(np.sum(np.maximum(c - 6, 0)))
    return int(np.sum(c == 2)), int(np.sum(c > 2)), cost


def _paths(t1, t2, log2b):
    """Per repetition, the chains of both operands under the window of least
    cost (lowest rotation on ties): [(two-row, longer) for A, for B]."""
    out = []
    for t in range(t1.shape[0]):
        best = None
        for s in range(0, min(log2b - LB, MAX_WINDOW) + 1):
            a, b = _chains(t1[t], log2b, s), _chains(t2[t], log2b, s)
            cost = a[2] + b[2]
            if best is None or cost < best[0]:
                best = (cost, (a[:2], b[:2]))
        out.append(best[1])
    return out


def test_two_row_chains_many_slots_f32_exact():
    n, ni, log2b, d = 8192, 48, 18, 3
    keys = draw_keys(9, 1000)[:d]
    t1, t2 = O.hash_tables(keys, n, n, log2b)
    paths = _paths(t1, t2, log2b)
    print("chains per repetition (two-row, longer) for A, B:", paths, flush=True)
    # at least one repetition has only two-row chains, more than 512 of
    # them in one operand: the path this test is for
    assert any(a[1] == 0 and b[1] == 0 and max(a[0], b[0]) > 512 for a, b in paths)
    announce(f"two-row chains over several slots f32 n={n} log2b={log2b}")
    T = torch()
    rng = np.random.default_rng(11)
    A = (rng.random((n, ni)) < 0.02) * rng.choice([-1.0, 1.0], size=(n, ni))
    B = (rng.random((ni, n)) < 0.02) * rng.choice([-1.0, 1.0], size=(ni, n))
    p_ref = O.bucket_sums(O.product(A, B), t1, t2, log2b)
    res = cmm.estimate(dev(A, T.float32), dev(B, T.float32), d, log2b, keys=keys, compute="f32",
                       dense=False)
    assert np.array_equal(host(res.p), p_ref)
