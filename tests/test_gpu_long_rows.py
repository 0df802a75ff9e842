"""Rows too long to be staged beside a transpose buffer (float64 rows of
about 4600 to 8600 elements, float32 rows of about 13700 to 17300): the
fused compress then transposes each operand through its own row area once
the step's rows are gathered.  Integer operands make every path exact, so p
must equal the oracle's bucket sums (Algorithm 1 Compress) bit for bit,
also where chains outnumber the descriptor slots (b_lo = b = 2^13) and at
the longest rows the layout takes."""
import numpy as np
import pytest

import oracle as O
import paper_2601_09477_amd as cmm
from workloads import draw_keys
from tests.gpu_util import announce, dev, host, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch().cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()


# (n_rows, n_inner, n_cols, log2b, d)
F64_SHAPES = [(6000, 300, 6000, 15, 3), (8200, 97, 5000, 14, 1), (8600, 64, 8600, 13, 3),
              (4700, 33, 8192, 16, 1)]


def _integer_case(shape, seed):
    nr, ni, nc, log2b, d = shape
    rng = np.random.default_rng(seed)
    A = rng.integers(-3, 4, size=(nr, ni)).astype(np.float64)
    B = rng.integers(-3, 4, size=(ni, nc)).astype(np.float64)
    keys = draw_keys(d, 7100 + seed)
    t1, t2 = O.hash_tables(keys, nr, nc, log2b)
    return A, B, keys, O.bucket_sums(O.product(A, B), t1, t2, log2b)


@pytest.mark.parametrize("shape", F64_SHAPES)
def test_long_rows_f64_bit_exact(shape):
    nr, ni, nc, log2b, d = shape
    announce(f"long rows f64 {shape}")
    A, B, keys, p_ref = _integer_case(shape, nr + nc)
    res = cmm.estimate(dev(A), dev(B), d, log2b, keys=keys)
    assert np.array_equal(host(res.p), p_ref)


def test_long_rows_f32_exact():
    # float32 rows of 15000 elements.  Sparse +-1 operands (2% nonzero) keep
    # every transform value below 300 in magnitude and every sum over k
    # below 2^24, so the float32 path is exact.
    shape = (15000, 48, 14000, 14, 3)
    nr, ni, nc, log2b, d = shape
    announce(f"long rows f32 {shape}")
    T = torch()
    rng = np.random.default_rng(5)
    A = (rng.random((nr, ni)) < 0.02) * rng.choice([-1.0, 1.0], size=(nr, ni))
    B = (rng.random((ni, nc)) < 0.02) * rng.choice([-1.0, 1.0], size=(ni, nc))
    keys = draw_keys(d, 7105)
    t1, t2 = O.hash_tables(keys, nr, nc, log2b)
    p_ref = O.bucket_sums(O.product(A, B), t1, t2, log2b)
    res = cmm.estimate(dev(A, T.float32), dev(B, T.float32), d, log2b, keys=keys, compute="f32")
    assert np.array_equal(host(res.p), p_ref)
