"""Rectangular products end to end (Section 2 notes that the method and the
implementation extend beyond square matrices): tall, wide and flat shapes
of some thousands of rows and columns through every compute path, against
the oracle's plain definition."""
import numpy as np
import pytest

import oracle as O
import paper_2601_09477_amd as cmm
from workloads import draw_keys
from tests.gpu_util import announce, dev, host, torch
from tests.numerics import f32_tolerance

pytestmark = pytest.mark.gpu

# (n_rows, n_inner, n_cols, log2b, d)
SHAPES = [(3000, 5000, 2000, 15, 5), (1024, 8192, 6000, 16, 3), (6000, 512, 700, 14, 3)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch().cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()


def _case(shape, integer, seed):
    nr, ni, nc, log2b, d = shape
    rng = np.random.default_rng(seed)
    if integer:
        A = rng.integers(-2, 3, size=(nr, ni)).astype(np.float64)
        B = rng.integers(-2, 3, size=(ni, nc)).astype(np.float64)
    else:
        A = rng.standard_normal((nr, ni))
        B = rng.standard_normal((ni, nc))
    keys = draw_keys(d, 4400 + seed)
    t1, t2 = O.hash_tables(keys, nr, nc, log2b)
    C = O.product(A, B)
    return A, B, keys, t1, t2, C


@pytest.mark.parametrize("shape", SHAPES)
def test_rectangular_f64_bit_exact(shape):
    nr, ni, nc, log2b, d = shape
    announce(f"rectangular f64 {shape}")
    A, B, keys, t1, t2, C = _case(shape, True, 1)
    p_ref = O.bucket_sums(C, t1, t2, log2b)
    res = cmm.estimate(dev(A), dev(B), d, log2b, keys=keys)
    assert np.array_equal(host(res.p), p_ref)
    rows = np.arange(0, nr, 37)
    assert np.array_equal(host(res.C_hat)[rows], O.extract(p_ref, t1, t2, "median", rows=rows))


@pytest.mark.parametrize("shape", SHAPES)
def test_rectangular_f32_fft_bf16(shape):
    nr, ni, nc, log2b, d = shape
    announce(f"rectangular f32 / fft / bf16 {shape}")
    T = torch()
    A, B, keys, t1, t2, C = _case(shape, False, 2)
    scale = np.linalg.norm(C) / ni
    # float32 transforms and sums: the tolerance derived in tests/numerics.py
    A32 = A.astype(np.float32).astype(np.float64)
    B32 = B.astype(np.float32).astype(np.float64)
    p32 = O.bucket_sums(O.product(A32, B32), t1, t2, log2b)
    res = cmm.estimate(dev(A, T.float32), dev(B, T.float32), d, log2b, keys=keys, compute="f32")
    assert np.abs(host(res.p) - p32).max() <= f32_tolerance(A32, B32, log2b, k_run=ni)
    # Pagh's FFT form in float64
    pc = O.bucket_sums_cyclic(C, t1, t2, log2b)
    res = cmm.estimate_fft(dev(A), dev(B), d, log2b, keys=keys)
    assert np.abs(host(res.p) - pc).max() <= 1e-9 * scale
    # the precision form (bf16 operands on the matrix cores): the rms error
    # of p within 8 eps rms(p) sqrt(n_inner) (see the precision tests)
    p_ref = O.bucket_sums(C, t1, t2, log2b)
    res = cmm.estimate(dev(A), dev(B), d, log2b, keys=keys, compute="bf16")
    dp = host(res.p) - p_ref
    rms = np.sqrt(np.mean(p_ref ** 2))
    assert np.sqrt(np.mean(dp ** 2)) <= 8 * 2.0 ** -8 * rms * np.sqrt(ni)
