"""Pins of the oracle's FFT form (Pagh's Compress / Decompress, Section 3.1):
the cyclic convolution against a hand-worked case, the two Compress routes
against each other, the plain definition against brute force and against
polynomial multiplication (identity tables), exact recovery with injective
tables, and unbiasedness / the variance bound over hash draws."""
import numpy as np
import pytest

import oracle as O
from workloads import draw_keys, small_random


def test_cyclic_convolution_hand_case():
    # b = 4: x0 y1 -> 1, x0 y3 -> 3, x1 y1 -> 2, x1 y3 -> 4 = 0 (mod 4)
    x = np.array([1.0, 2.0, 0.0, 0.0])
    y = np.array([0.0, 1.0, 0.0, 3.0])
    assert O.cyclic_convolution(x, y).tolist() == [6.0, 1.0, 2.0, 3.0]
    # convolution theorem (numpy's transform as the library routine)
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal(16), rng.standard_normal(16)
    via_fft = np.fft.ifft(np.fft.fft(x) * np.fft.fft(y)).real
    assert np.abs(O.cyclic_convolution(x, y) - via_fft).max() < 1e-12


def _tabs(idx_h, signs):
    return ((np.asarray(idx_h, dtype=np.uint32)) |
            (np.asarray(signs, dtype=np.uint32) << np.uint32(31)))[None, :]


def test_identity_tables_give_polynomial_product():
    # h1(i) = i, h2(j) = j, positive signs, b >= n_rows + n_cols - 1: the
    # cyclic bucket sums are the polynomial product sum_k a_k(z) b_k(z)
    rng = np.random.default_rng(1)
    nr, ni, nc, log2b = 9, 5, 6, 4
    A = rng.standard_normal((nr, ni))
    B = rng.standard_normal((ni, nc))
    t1 = _tabs(np.arange(nr), np.zeros(nr))
    t2 = _tabs(np.arange(nc), np.zeros(nc))
    want = np.zeros(1 << log2b)
    for k in range(ni):
        c = np.convolve(A[:, k], B[k, :])
        want[:len(c)] += c
    got = O.bucket_sums_cyclic(O.product(A, B), t1, t2, log2b)[0]
    assert np.abs(got - want).max() < 1e-12
    assert np.abs(O.compress_fft(A, B, t1, t2, log2b)[0] - want).max() < 1e-12
    # (the xor form differs: bucket 3 collects i xor j = 3 instead of i + j = 3)
    assert np.abs(O.bucket_sums(O.product(A, B), t1, t2, log2b)[0] - want).max() > 1e-3


def test_injective_tables_recover_product():
    # h1(i) = i, h2(j) = 8 j with b = 8 * 8: every (i, j) has its own bucket
    # (i + 8 j), so Decompress returns C exactly, with any signs
    rng = np.random.default_rng(2)
    A = rng.integers(-4, 5, (8, 7)).astype(float)
    B = rng.integers(-4, 5, (7, 8)).astype(float)
    C = A @ B
    t1 = np.vstack([_tabs(np.arange(8), rng.integers(0, 2, 8)) for _ in range(3)])
    t2 = np.vstack([_tabs(8 * np.arange(8), rng.integers(0, 2, 8)) for _ in range(3)])
    p = O.bucket_sums_cyclic(C, t1, t2, 6)
    assert np.array_equal(O.extract_cyclic(p, t1, t2, "median"), C)
    assert np.array_equal(O.extract_cyclic(p, t1, t2, "mean"), C)


def test_extract_cyclic_wrapping_tables_recover_product():
    # h1(i) = 40 + i, h2(j) = (30 + 8 j) mod 64 with b = 64: the sums
    # h1 + h2 = 70 + i + 8 j carry past b and wrap, and (h1 + h2) mod b =
    # 6 + i + 8 j (mod 64) is injective over the 8 x 8 entries, so
    # Decompress of the cyclic bucket sums returns C exactly.  Gathering at
    # h1 xor h2 or at the unwrapped sum would not (checked below), so this
    # pins the index of Pagh's Decompress, h = h1 + h2 mod b (Section 3.1).
    rng = np.random.default_rng(12)
    A = rng.integers(-4, 5, (8, 6)).astype(float)
    B = rng.integers(-4, 5, (6, 8)).astype(float)
    C = A @ B
    h1 = 40 + np.arange(8)
    h2 = (30 + 8 * np.arange(8)) % 64
    t1 = np.vstack([_tabs(h1, rng.integers(0, 2, 8)) for _ in range(3)])
    t2 = np.vstack([_tabs(h2, rng.integers(0, 2, 8)) for _ in range(3)])
    p = O.bucket_sums_cyclic(C, t1, t2, 6)
    assert np.array_equal(O.extract_cyclic(p, t1, t2, "median"), C)
    assert np.array_equal(O.extract_cyclic(p, t1, t2, "mean"), C)
    # the mutations a wrong index would make fail to recover C
    s = O.sign(t1[0])[:, None] * O.sign(t2[0])[None, :]
    xor_idx = h1[:, None] ^ h2[None, :]
    assert not np.array_equal(s * p[0][xor_idx], C)
    assert ((h1[:, None] + h2[None, :]) >= 64).any()      # the unwrapped sum leaves the table


def test_extract_cyclic_against_entrywise_loop():
    # tables whose sums carry and wrap (b = 64): h1(i) = 40 + i, h2(j) = 30 + 5 j;
    # the estimate of every entry from its own loop over repetitions, with
    # Python integers for the bucket and the median as the middle of the sorted values
    rng = np.random.default_rng(13)
    d, nr, nc, b = 5, 9, 7, 64
    h1 = 40 + np.arange(nr)
    h2 = (30 + 5 * np.arange(nc)) % b
    t1 = np.vstack([_tabs(h1, rng.integers(0, 2, nr)) for _ in range(d)])
    t2 = np.vstack([_tabs(h2, rng.integers(0, 2, nc)) for _ in range(d)])
    p = rng.standard_normal((d, b))
    med = O.extract_cyclic(p, t1, t2, "median")
    mean = O.extract_cyclic(p, t1, t2, "mean")
    for i in range(nr):
        for j in range(nc):
            vals = []
            for t in range(d):
                bucket = (int(h1[i]) + int(h2[j])) % b
                sgn = (-1.0 if t1[t][i] >> 31 else 1.0) * (-1.0 if t2[t][j] >> 31 else 1.0)
                vals.append(sgn * p[t][bucket])
            assert med[i, j] == sorted(vals)[d // 2]
            assert abs(mean[i, j] - sum(vals) / d) <= 1e-15 * max(1.0, max(map(abs, vals)))


def test_plain_definition_brute_force():
    w = small_random(7, 4, 5, 3, 2, seed=3, integer=True)
    t1, t2 = O.hash_tables(w.keys, 7, 5, 3)
    C = O.product(w.A, w.B)
    want = np.zeros((2, 8))
    for t in range(2):
        for i in range(7):
            for j in range(5):
                x = (int(O.bucket(t1[t][i])) + int(O.bucket(t2[t][j]))) % 8
                want[t, x] += O.sign(t1[t][i]) * O.sign(t2[t][j]) * C[i, j]
    assert np.array_equal(O.bucket_sums_cyclic(C, t1, t2, 3), want)


@pytest.mark.parametrize("integer", [True, False])
def test_fft_route_equals_plain_definition(integer):
    w = small_random(60, 45, 50, 9, 3, seed=4, integer=integer)
    t1, t2 = O.hash_tables(w.keys, 60, 50, 9)
    p_fft = O.compress_fft(w.A, w.B, t1, t2, 9, k_chunk=16)
    p_def = O.bucket_sums_cyclic(O.product(w.A, w.B), t1, t2, 9)
    scale = np.abs(p_def).max()
    assert np.abs(p_fft - p_def).max() <= 1e-12 * scale
    if integer:
        assert np.array_equal(np.rint(p_fft), p_def)


def test_cyclic_estimator_unbiased_with_variance_bound():
    # Pagh's Theorem 3.1: each repetition is unbiased with variance at most
    # ||C||_F^2 / b over the hash draw
    rng = np.random.default_rng(5)
    A = rng.standard_normal((12, 10))
    B = rng.standard_normal((10, 14))
    C = A @ B
    log2b, draws = 5, 3000
    keys = draw_keys(draws, 123)
    t1, t2 = O.hash_tables(keys, 12, 14, log2b)
    p = O.bucket_sums_cyclic(C, t1, t2, log2b)
    i, j = 3, 7
    # each draw's estimate through Decompress itself (one repetition at a time)
    x = np.array([O.extract_cyclic(p[t:t + 1], t1[t:t + 1], t2[t:t + 1], "median")[i, j]
                  for t in range(draws)])
    bound = (np.linalg.norm(C) ** 2 - C[i, j] ** 2) / (1 << log2b)
    assert abs(x.mean() - C[i, j]) <= 4 * np.sqrt(bound / draws)
    assert x.var() <= 1.25 * bound
