"""Pins for the CPU oracle: each check compares the oracle with something
other than itself (hand-worked values, closed forms, brute force, library
routines, invariants of the mathematics)."""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import oracle as O
from workloads import (draw_keys, draw_tabulation_keys, exact_sparse_256, hadamard_sparse,
                       small_random)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _tables(h, s, log2b):
    """Build table entries from explicit buckets and signs (no hashing)."""
    h = np.asarray(h, dtype=np.uint32)
    s = np.asarray(s)
    return (h | np.where(s < 0, np.uint32(1 << 31), np.uint32(0))).astype(np.uint32)[None, :]


# ---------------------------------------------------------------------- hash
def test_hash_golden():
    g = _load("hash_small.json")
    for case in g["cases"]:
        got = O.multiply_add_shift(int(case["a"]), int(case["c"]), np.array(case["x"]), case["log2b"])
        assert got.tolist() == case["h"], case


@pytest.mark.parametrize("m", [1, 4, 12, 16, 18, 31])
def test_hash_identity_special_case(m):
    # a = 2^(64-m), c = 0  =>  h(x) = x mod 2^m  (the shift undoes the multiply)
    x = np.arange(0, 5000, 7, dtype=np.uint64)
    got = O.multiply_add_shift(1 << (64 - m), 0, x, m)
    assert np.array_equal(got, x % (1 << m))


def test_hash_constant_and_wrap():
    x = np.arange(100, dtype=np.uint64)
    # a = 0: constant bucket c >> (64 - m)
    assert np.all(O.multiply_add_shift(0, 0xDEADBEEF00000000, x, 8) == (0xDEADBEEF00000000 >> 56))
    # a = 2^64 - 1 (i.e. -1): (-x mod 2^64) >> (64 - m) = 2^m - 1 for 1 <= x < 2^(64-m)
    got = O.multiply_add_shift((1 << 64) - 1, 0, x[1:], 10)
    assert np.all(got == (1 << 10) - 1)
    # sign hash with a = 2^63: top bit = x & 1
    assert np.array_equal(O.multiply_add_shift(1 << 63, 0, x, 1), x & 1)


def test_hash_tables_encoding_matches_python_ints():
    keys = draw_keys(3, 99)
    t1, t2 = O.hash_tables(keys, 300, 200, 13)
    for t in range(3):
        (a1, c1), (a2, c2), (as1, cs1), (as2, cs2) = [(int(k[0]), int(k[1])) for k in keys[t]]
        for i in (0, 1, 17, 299):
            v = (a1 * i + c1) % (1 << 64)
            sv = (as1 * i + cs1) % (1 << 64)
            assert int(t1[t, i]) == (v >> 51) | ((sv >> 63) << 31)
        for j in (0, 5, 199):
            v = (a2 * j + c2) % (1 << 64)
            sv = (as2 * j + cs2) % (1 << 64)
            assert int(t2[t, j]) == (v >> 51) | ((sv >> 63) << 31)


@pytest.mark.slow
def test_hash_pairwise_collisions_theorem1():
    # Theorem 1: h(i,j) = h1(i) xor h2(j) is 2-wise independent, so two
    # distinct pairs collide with probability 1/b.  Estimate over key draws.
    log2b, draws = 6, 4000
    b = 1 << log2b
    hits = np.zeros(3)
    pairs = [((0, 0), (1, 0)), ((0, 0), (0, 1)), ((2, 3), (5, 7))]
    for s in range(draws):
        t1, t2 = O.hash_tables(draw_keys(1, 50_000 + s), 8, 8, log2b)
        h1, h2 = O.bucket(t1[0]), O.bucket(t2[0])
        for q, ((i, j), (k, l)) in enumerate(pairs):
            hits[q] += (h1[i] ^ h2[j]) == (h1[k] ^ h2[l])
    rate = hits / draws
    # binomial sd at p=1/64, N=4000 is ~0.002; allow 4 sd
    assert np.all(np.abs(rate - 1 / b) < 4 * np.sqrt((1 / b) * (1 - 1 / b) / draws)), rate


def test_hash_uniformity_chi_square():
    log2b = 8
    t1, _ = O.hash_tables(draw_keys(1, 4242), 1 << 16, 1, log2b)
    counts = np.bincount(O.bucket(t1[0]), minlength=1 << log2b)
    expected = (1 << 16) / (1 << log2b)
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 255 + 6 * np.sqrt(2 * 255)   # mean dof, +6 sd
    signs = O.sign(t1[0])
    assert abs(signs.mean()) < 0.02


# ------------------------------------------------- alternative hash families
@pytest.mark.parametrize("m", [1, 5, 13, 16, 31])
def test_multiply_shift_special_cases(m):
    x = np.arange(0, 70000, 13, dtype=np.uint64)
    # a = 2^(64-m) + 1 (odd): a x = x 2^(64-m) + x, whose top m bits are x mod 2^m
    assert np.array_equal(O.multiply_shift((1 << (64 - m)) + 1, x, m), x % (1 << m))
    # the drawn word's low bit is forced to one: 2^(64-m) behaves as 2^(64-m) + 1
    assert np.array_equal(O.multiply_shift(1 << (64 - m), x, m), x % (1 << m))
    # no additive term: x = 0 always hashes to 0
    assert O.multiply_shift(0x9E3779B97F4A7C15, np.zeros(1, np.uint64), m)[0] == 0
    # a = 2^64 - 1: (-x mod 2^64) >> (64 - m) = 2^m - 1 for 1 <= x < 2^(64-m)
    assert np.all(O.multiply_shift((1 << 64) - 1, x[1:], m) == (1 << m) - 1)


@pytest.mark.slow
def test_multiply_shift_universal():
    # Dietzfelbinger et al.: two distinct keys collide with probability at
    # most 2 / b over the odd multipliers
    log2b, draws = 6, 4000
    keys = draw_keys(draws, 777)
    hits = np.zeros(3)
    pairs = [(1, 2), (3, 1000), (12345, 54321)]
    for s in range(draws):
        h = O.multiply_shift(int(keys[s, 0, 0]), np.array([1, 2, 3, 1000, 12345, 54321], np.uint64),
                             log2b)
        hits += [h[0] == h[1], h[2] == h[3], h[4] == h[5]]
    rate = hits / draws
    bound = 2 / (1 << log2b)
    assert np.all(rate <= bound + 4 * np.sqrt(bound * (1 - bound) / draws)), rate


def test_tabulation_byte_order_closed_form():
    # T[q][v] = v << (56 - 8 q) puts byte q of x into bits [56 - 8q, 64 - 8q):
    # the 32 top bits of h(x) are x with its bytes reversed
    T = np.array([[v << (56 - 8 * q) for v in range(256)] for q in range(4)], dtype=np.uint64)
    x = np.array([0, 1, 0xFF, 0x100, 0x12345678, 0xDEADBEEF, 0xFFFFFFFF], dtype=np.uint64)
    bswap = [int.from_bytes(int(v).to_bytes(4, "little"), "big") for v in x]
    assert O.tabulation(T, x, 32).tolist() == bswap
    # with one output bit the hash is bit 63 of the word: bit 7 of byte 0 of x
    assert O.tabulation(T, x, 1).tolist() == [(int(v) >> 7) & 1 for v in x]


def test_tabulation_xor_structure():
    # h is an xor of per-byte table words: for keys that differ crosswise in
    # two byte positions (a rectangle), the four full 64-bit hashes xor to 0,
    # while a key pair that differs in one byte changes h by the xor of the
    # two table words of that byte
    T = draw_tabulation_keys(1, 31)[0, 0]
    rng = np.random.default_rng(5)
    for _ in range(50):
        base = int(rng.integers(0, 1 << 32))
        q1, q2 = rng.choice(4, 2, replace=False)
        v1, v2 = rng.integers(0, 256, 2)

        def put(x, q, v):
            return (x & ~(0xFF << (8 * q))) | (int(v) << (8 * q))
        xs = np.array([base, put(base, q1, v1), put(base, q2, v2), put(put(base, q1, v1), q2, v2)],
                      dtype=np.uint64)
        h = O.tabulation(T, xs, 64)
        assert h[0] ^ h[1] ^ h[2] ^ h[3] == 0
        b0 = (base >> (8 * q1)) & 0xFF
        assert h[0] ^ h[1] == T[q1][b0] ^ T[q1][int(v1)]


def test_tabulation_uniform_and_pairwise():
    log2b = 8
    keys = draw_tabulation_keys(1, 4242)
    t1, _ = O.hash_tables_family("tabulation", keys, 1 << 16, 1, log2b)
    counts = np.bincount(O.bucket(t1[0]), minlength=1 << log2b)
    expected = (1 << 16) / (1 << log2b)
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 255 + 6 * np.sqrt(2 * 255)
    assert abs(O.sign(t1[0]).mean()) < 0.02
    # collisions of a fixed pair of keys over independent tables: rate 1 / b
    draws, b = 3000, 1 << 6
    keys = draw_tabulation_keys(draws, 99)
    hits = sum(O.tabulation(keys[s, 0], np.array([7, 70000], np.uint64), 6).tolist()[0] ==
               O.tabulation(keys[s, 0], np.array([7, 70000], np.uint64), 6).tolist()[1]
               for s in range(draws))
    assert abs(hits / draws - 1 / b) < 4 * np.sqrt((1 / b) * (1 - 1 / b) / draws)


def test_family_tables_layout():
    # which drawn function feeds which field: zero bucket tables and a sign
    # table that is all ones give bucket 0 and sign -1 for every index
    keys = np.zeros((2, 4, 4, 256), dtype=np.uint64)
    keys[:, 2] = np.uint64(1 << 63)          # s1: top bit set for every byte value
    keys[:, 2, 1:] = 0                       # ... from byte 0 only (odd count of set words)
    keys[1, 1, 0, :] = np.arange(256, dtype=np.uint64) << np.uint64(56)   # h2 of t = 1
    t1, t2 = O.hash_tables_family("tabulation", keys, 40, 300, 8)
    assert np.all(t1 == np.uint32(1 << 31))
    assert np.all(t2[0] == 0)
    assert np.array_equal(t2[1], (np.arange(300) & 0xFF).astype(np.uint32))
    # the multiply-add-shift entry is the Section 4.2 table builder
    k = draw_keys(3, 8)
    for a, b in zip(O.hash_tables_family("multiply_add_shift", k, 50, 60, 11),
                    O.hash_tables(k, 50, 60, 11)):
        assert np.array_equal(a, b)
    # multiply-shift reads the first word of each pair only
    k2 = k.copy()
    k2[:, :, 1] = 0
    for a, b in zip(O.hash_tables_family("multiply_shift", k, 50, 60, 11),
                    O.hash_tables_family("multiply_shift", k2, 50, 60, 11)):
        assert np.array_equal(a, b)


# ------------------------------------------------------------------ transform
def test_wht_golden_and_matrix():
    g = _load("wht_h4.json")
    assert O.wht(np.array(g["x"], float)).tolist() == g["Hx"]
    assert O.wht_matrix(2).tolist() == g["H"]


@pytest.mark.parametrize("m", [1, 3, 6, 9])
def test_wht_matches_scipy_hadamard_and_definition(m):
    b = 1 << m
    H = scipy.linalg.hadamard(b).astype(float)     # Sylvester construction
    assert np.array_equal(O.wht_matrix(m), H)
    rng = np.random.default_rng(m)
    x = rng.integers(-50, 50, size=(3, b)).astype(float)
    assert np.array_equal(O.wht(x), x @ H.T)
    # basis vector e_r -> row r of H (symmetric)
    for r in (0, 1, b - 1, b // 3):
        e = np.zeros(b); e[r] = 1
        assert np.array_equal(O.wht(e), H[r])


@pytest.mark.parametrize("m", [4, 10, 16])
def test_wht_self_inverse_up_to_b(m):
    rng = np.random.default_rng(100 + m)
    x = rng.integers(-1000, 1000, size=(2, 1 << m)).astype(float)
    assert np.array_equal(O.wht(O.wht(x)), (1 << m) * x)            # H H = b I (exact on integers)
    assert np.array_equal(O.wht(O.wht(x), 2.0 ** -m), x)
    y = rng.standard_normal(1 << m)
    assert np.isclose(np.sum(O.wht(y) ** 2), (1 << m) * np.sum(y ** 2))   # Parseval


def test_xor_convolution_golden_and_theorem():
    g = _load("xor_conv_4.json")
    x, y = np.array(g["x"], float), np.array(g["y"], float)
    assert O.xor_convolution(x, y).tolist() == g["z"]
    rng = np.random.default_rng(7)
    for m in (1, 4, 7):
        x = rng.integers(-9, 10, 1 << m).astype(float)
        y = rng.integers(-9, 10, 1 << m).astype(float)
        brute = np.array([sum(x[i] * y[i ^ k] for i in range(1 << m)) for k in range(1 << m)])
        via_wht = O.wht(O.wht(x) * O.wht(y), 2.0 ** -m)
        assert np.array_equal(via_wht, brute)
        assert np.array_equal(O.xor_convolution(x, y), brute)


# ------------------------------------------------------------------ sketching
def test_count_sketch_against_dense_sketch_matrix():
    rng = np.random.default_rng(3)
    A = rng.integers(-5, 6, size=(40, 12)).astype(float)
    B = rng.integers(-5, 6, size=(12, 30)).astype(float)
    log2b = 5
    t1, t2 = O.hash_tables(draw_keys(2, 77), 40, 30, log2b)
    for t in range(2):
        S1 = np.zeros((32, 40)); S1[O.bucket(t1[t]), np.arange(40)] = O.sign(t1[t])
        S2 = np.zeros((32, 30)); S2[O.bucket(t2[t]), np.arange(30)] = O.sign(t2[t])
        got_a = O.count_sketch(A, t1, 0, 3, 7, log2b)[t]      # [kc][b]
        got_b = O.count_sketch(B, t2, 1, 3, 7, log2b)[t]
        assert np.array_equal(got_a, (S1 @ A[:, 3:10]).T)
        assert np.array_equal(got_b, (S2 @ B[3:10, :].T).T)


def test_accumulate_is_sum_of_products():
    rng = np.random.default_rng(4)
    X = rng.integers(-9, 9, (2, 5, 8)).astype(float)
    Y = rng.integers(-9, 9, (2, 5, 8)).astype(float)
    want = np.einsum("tku,tku->tu", X, Y)
    assert np.array_equal(O.accumulate(X, Y), want)


# ------------------------------------------------------------------- compress
def test_pipeline_golden_2x2():
    g = _load("pipeline_2x2.json")
    A, B = np.array(g["A"], float), np.array(g["B"], float)
    for case in g["cases"]:
        t1 = _tables(case["h1"], case["s1"], g["log2b"])
        t2 = _tables(case["h2"], case["s2"], g["log2b"])
        p_alg1 = O.compress_alg1(A, B, t1, t2, g["log2b"])
        p_def = O.bucket_sums(O.product(A, B), t1, t2, g["log2b"])
        assert p_alg1[0].tolist() == case["p"], case["name"]
        assert p_def[0].tolist() == case["p"], case["name"]
        assert O.extract(p_def, t1, t2, "median").tolist() == case["C_hat"]


def test_alg1_route_equals_bucket_sums_integer_exact():
    w = small_random(48, 40, 56, 7, 3, seed=11, integer=True)
    t1, t2 = O.hash_tables(w.keys, 48, 56, 7)
    p1 = O.compress_alg1(w.A, w.B, t1, t2, 7, k_chunk=16)
    p2 = O.bucket_sums(O.product(w.A, w.B), t1, t2, 7)
    assert np.array_equal(p1, p2)


def test_alg1_route_equals_bucket_sums_real():
    w = small_random(64, 50, 64, 9, 5, seed=12)
    t1, t2 = O.hash_tables(w.keys, 64, 64, 9)
    p1 = O.compress_alg1(w.A, w.B, t1, t2, 9)
    C = O.product(w.A, w.B)
    p2 = O.bucket_sums(C, t1, t2, 9)
    assert np.max(np.abs(p1 - p2)) <= 1e-13 * np.linalg.norm(C) / 64 * 64


def test_identity_hash_reduces_to_matmul():
    # h1(i) = i * n, h2(j) = j, signs +1, b = n^2: h1 xor h2 = i n + j is
    # injective, so p[i n + j] = C[i, j] and the estimate equals A B exactly.
    n = 8
    rng = np.random.default_rng(5)
    A = rng.integers(-20, 20, (n, n)).astype(float)
    B = rng.integers(-20, 20, (n, n)).astype(float)
    log2b = 6
    t1 = _tables(np.arange(n) * n, np.ones(n), log2b).repeat(3, 0)
    t2 = _tables(np.arange(n), np.ones(n), log2b).repeat(3, 0)
    brute = np.array([[sum(int(A[i, k]) * int(B[k, j]) for k in range(n)) for j in range(n)]
                      for i in range(n)], dtype=float)
    p = O.compress_alg1(A, B, t1, t2, log2b)
    assert np.array_equal(p[0].reshape(n, n), brute)
    assert np.array_equal(O.extract(p, t1, t2, "median"), brute)
    assert np.array_equal(O.extract(p, t1, t2, "mean"), brute)


def test_topk_against_brute_force_on_exact_tables():
    # Injective tables make Decompress return C = A B exactly (as above), so
    # the top-k entries are those of C: brute force over every entry with
    # Python integers, ordered by magnitude and then by the row-major index.
    # Small integer entries give many ties, which the index order decides.
    n = 8
    rng = np.random.default_rng(17)
    A = rng.integers(-3, 4, (n, n)).astype(float)
    B = rng.integers(-3, 4, (n, n)).astype(float)
    log2b = 6
    t1 = _tables(np.arange(n) * n, rng.integers(0, 2, n), log2b).repeat(3, 0)
    t2 = _tables(np.arange(n), rng.integers(0, 2, n), log2b).repeat(3, 0)
    p = O.bucket_sums(O.product(A, B), t1, t2, log2b)
    C = [[sum(int(A[i, q]) * int(B[q, j]) for q in range(n)) for j in range(n)] for i in range(n)]
    ranked = sorted(((-abs(C[i][j]), i * n + j) for i in range(n) for j in range(n)))
    for k in (1, 5, 17, n * n):
        rows, cols, vals = O.extract_topk(p, t1, t2, k, "median")
        want = ranked[:k]
        assert [int(r) * n + int(c) for r, c in zip(rows, cols)] == [ix for _, ix in want]
        assert [float(v) for v in vals] == [float(C[ix // n][ix % n]) for _, ix in want]
    assert len({abs(C[i][j]) for i in range(n) for j in range(n)}) < n * n   # ties occur


def test_bucket_sums_sparse_equals_dense_definition():
    # the nonzero-entry form of the bucket sums against the dense form on a
    # sparse product, and against brute force over the entries
    rng = np.random.default_rng(4)
    n_rows, n_cols, log2b = 40, 30, 6
    C = np.zeros((n_rows, n_cols))
    pos = rng.choice(n_rows * n_cols, size=50, replace=False)
    C.flat[pos] = rng.standard_normal(50)
    t1, t2 = O.hash_tables(draw_keys(3, 61), n_rows, n_cols, log2b)
    r, c = np.nonzero(C)
    ps = O.bucket_sums_sparse(r, c, C[r, c], t1, t2, log2b)
    pd = O.bucket_sums(C, t1, t2, log2b)
    assert np.allclose(ps, pd, rtol=0, atol=1e-14)
    brute = np.zeros_like(ps)
    for t in range(3):
        for i, j in zip(r, c):
            x = (int(t1[t][i]) & 63) ^ (int(t2[t][j]) & 63)
            sg = (-1.0 if t1[t][i] >> 31 else 1.0) * (-1.0 if t2[t][j] >> 31 else 1.0)
            brute[t, x] += sg * C[i, j]
    assert np.allclose(ps, brute, rtol=0, atol=1e-14)


def test_extract_entries_equals_dense_extract():
    # the list form of Decompress against the dense form at the same entries
    w = small_random(30, 20, 25, 7, 5, seed=8)
    t1, t2 = O.hash_tables(w.keys, 30, 25, 7)
    p = O.bucket_sums(O.product(w.A, w.B), t1, t2, 7)
    rng = np.random.default_rng(2)
    rows, cols = rng.integers(0, 30, 40), rng.integers(0, 25, 40)
    for est in ("median", "mean"):
        dense = O.extract(p, t1, t2, est)
        assert np.array_equal(O.extract_entries(p, t1, t2, rows, cols, est), dense[rows, cols])
    out = O.extract_entries(p, t1, t2, [-1, 30, 3], [0, 0, 25])
    assert np.all(np.isnan(out))


def test_bucket_sums_brute_force_tiny():
    rng = np.random.default_rng(6)
    C = rng.integers(-9, 9, (5, 6)).astype(float)
    t1, t2 = O.hash_tables(draw_keys(2, 31), 5, 6, 3)
    p = O.bucket_sums(C, t1, t2, 3)
    for t in range(2):
        want = np.zeros(8)
        for i in range(5):
            for j in range(6):
                x = (int(t1[t, i]) & 7) ^ (int(t2[t, j]) & 7)
                s = (-1 if t1[t, i] >> 31 else 1) * (-1 if t2[t, j] >> 31 else 1)
                want[x] += s * C[i, j]
        assert np.array_equal(p[t], want)


def test_exact_recovery_thm34_regime():
    # b >= 8 nnz(C), d >= 6 log2 n: every entry recovered (Section 5.6).
    n, nnz, log2b, d = 64, 8, 10, 37
    rng = np.random.default_rng(8)
    A, B, C_exact = hadamard_sparse(n, nnz, rng)
    C_hat, p, t1, t2 = O.estimate(A, B, draw_keys(d, 123), log2b)
    tol = 1e-12 * np.linalg.norm(C_exact) / n
    assert np.max(np.abs(C_hat - C_exact)) <= tol


def test_hadamard_workload_product_is_sparse():
    w = exact_sparse_256(0)
    C = O.product(w.A, w.B)
    assert np.max(np.abs(C - w.C_exact)) < 1e-10
    assert np.count_nonzero(w.C_exact) == 256


def test_metamorphic_invariants():
    w = small_random(32, 24, 40, 8, 5, seed=13, integer=True)
    t1, t2 = O.hash_tables(w.keys, 32, 40, 8)
    C = O.product(w.A, w.B)
    p = O.bucket_sums(C, t1, t2, 8)
    C_hat = O.extract(p, t1, t2, "median")
    # transpose symmetry: (B^T, A^T) with the roles of the tables swapped gives C_hat^T
    pT = O.bucket_sums(O.product(w.B.T, w.A.T), t2, t1, 8)
    assert np.array_equal(O.extract(pT, t2, t1, "median"), C_hat.T)
    # flipping every sign of s1 and of s2 leaves the estimate unchanged
    f1, f2 = t1 ^ np.uint32(1 << 31), t2 ^ np.uint32(1 << 31)
    assert np.array_equal(O.extract(O.bucket_sums(C, f1, f2, 8), f1, f2, "median"), C_hat)
    # XOR-shifting both bucket hashes by the same delta leaves it unchanged
    g1, g2 = t1 ^ np.uint32(0x5A), t2 ^ np.uint32(0x5A)
    assert np.array_equal(O.extract(O.bucket_sums(C, g1, g2, 8), g1, g2, "median"), C_hat)
    # the mean estimator is linear in A
    A2 = w.A * 3 - 1
    m1 = O.extract(O.bucket_sums(O.product(w.A, w.B), t1, t2, 8), t1, t2, "mean")
    m2 = O.extract(O.bucket_sums(O.product(A2, w.B), t1, t2, 8), t1, t2, "mean")
    m3 = O.extract(O.bucket_sums(O.product(w.A + A2, w.B), t1, t2, 8), t1, t2, "mean")
    assert np.allclose(m1 + m2, m3, atol=1e-9)


def test_median_matches_sorted_middle():
    rng = np.random.default_rng(9)
    p = rng.standard_normal((7, 64))
    t1, t2 = O.hash_tables(draw_keys(7, 3), 10, 12, 6)
    got = O.extract(p, t1, t2, "median")
    x = O.gather_reps(p, t1, t2, np.arange(10), np.arange(12))
    assert np.array_equal(got, np.sort(x, axis=0)[3])
    with pytest.raises(ValueError):
        O.extract(p[:6], t1[:6], t2[:6], "median")


@pytest.mark.slow
def test_unbiased_and_variance_bound():
    # Section 3.1 / 5.3: with d = 1 the estimate is unbiased with variance
    # at most ||C||_F^2 / b.  1000 independent hash draws at n = 32.
    n, log2b, draws = 32, 6, 1000
    rng = np.random.default_rng(10)
    A = rng.standard_normal((n, n)); B = rng.standard_normal((n, n))
    C = A @ B
    i, j = 3, 5
    ests = []
    for s in range(draws):
        t1, t2 = O.hash_tables(draw_keys(1, 10_000 + s), n, n, log2b)
        p = O.bucket_sums(C, t1, t2, log2b)
        ests.append(O.extract(p, t1, t2, "median", rows=[i], cols=[j])[0, 0])
    ests = np.array(ests)
    bound = np.sum(C ** 2) / (1 << log2b)
    assert abs(ests.mean() - C[i, j]) < 4 * np.sqrt(bound / draws)
    assert ests.var() <= 1.2 * bound


# ------------------------------------------------------------------- gradient
def test_gradient_closed_form_vs_finite_differences():
    # L is bilinear in (A, B) for fixed hashes, so central differences are
    # exact up to rounding.
    n_r, n_i, n_c, log2b, d = 12, 10, 14, 6, 3
    rng = np.random.default_rng(14)
    A = rng.standard_normal((n_r, n_i)); B = rng.standard_normal((n_i, n_c))
    W = rng.standard_normal((n_r, n_c))
    t1, t2 = O.hash_tables(draw_keys(d, 555), n_r, n_c, log2b)

    def loss(A_, B_):
        p = O.bucket_sums(O.product(A_, B_), t1, t2, log2b)
        return np.sum(W * O.extract(p, t1, t2, "mean"))

    dA, dB, _ = O.grad_mean(A, B, W, t1, t2, log2b)
    h = 1e-3
    for (i, k) in [(0, 0), (3, 7), (11, 9), (5, 2)]:
        Ap, Am = A.copy(), A.copy(); Ap[i, k] += h; Am[i, k] -= h
        fd = (loss(Ap, B) - loss(Am, B)) / (2 * h)
        assert abs(fd - dA[i, k]) <= 1e-9 * (1 + abs(fd))
    for (k, j) in [(0, 0), (9, 13), (4, 6)]:
        Bp, Bm = B.copy(), B.copy(); Bp[k, j] += h; Bm[k, j] -= h
        fd = (loss(A, Bp) - loss(A, Bm)) / (2 * h)
        assert abs(fd - dB[k, j]) <= 1e-9 * (1 + abs(fd))


def test_gradient_brute_force_jacobian():
    # dL/dC[i,j] computed by perturbing C directly (the estimator is linear in C).
    n, log2b, d = 6, 4, 3
    rng = np.random.default_rng(15)
    W = rng.standard_normal((n, n))
    t1, t2 = O.hash_tables(draw_keys(d, 777), n, n, log2b)
    _, _, G = O.grad_mean(np.eye(n), np.eye(n), W, t1, t2, log2b)
    for i in range(n):
        for j in range(n):
            E = np.zeros((n, n)); E[i, j] = 1.0
            est = O.extract(O.bucket_sums(E, t1, t2, log2b), t1, t2, "mean")
            assert np.isclose(np.sum(W * est), G[i, j], atol=1e-12)
