"""The evaluation protocol on the CPU: the instance families of Section 5.2
pinned against their closed-form products, and the oracle's correctness
counters (Section 5.4) and per-repetition values against hand-worked cases
and the definitions they restate."""
import math

import numpy as np
import pytest

import oracle as O
from workloads import draw_keys, small_random
from workloads import instances as I


def _np(x):
    return x.detach().cpu().numpy()


@pytest.mark.parametrize("seed", [0, 1])
def test_logunit_product_closed_form(seed):
    n = 256
    w = I.logunit(n, seed)
    C = _np(w.A) @ _np(w.B)
    want = np.zeros((n, n))
    want[_np(w.C_rows), _np(w.C_cols)] = _np(w.C_vals)
    assert np.abs(C - want).max() <= 1e-10
    # log2 n entries 1, one non-zero per row and column, the rest 1e-4
    assert np.count_nonzero(np.isclose(want, 1.0)) == int(math.log2(n))
    assert np.array_equal(np.sort(_np(w.C_cols)), np.arange(n))
    assert np.all(np.isclose(want[_np(w.big_rows), _np(w.big_cols)], 1.0))
    assert np.count_nonzero(np.isclose(want, 1e-4)) == n - int(math.log2(n))


@pytest.mark.parametrize("seed", [0, 3])
def test_diagonal_product_closed_form(seed):
    n = 128
    w = I.diagonal(n, seed)
    C = _np(w.A) @ _np(w.B)
    want = np.zeros((n, n))
    want[_np(w.C_rows), _np(w.C_cols)] = _np(w.C_vals)
    assert np.abs(C - want).max() <= 1e-12
    v = np.abs(_np(w.C_vals))
    assert np.all((v >= 0.5) & (v < 1.0))
    assert len(_np(w.big_rows)) == n


def test_covariance_planted_pair():
    n = 1024
    vals, bg = [], []
    for seed in range(6):
        w = I.covariance(n, seed)
        C = _np(w.A) @ _np(w.B)
        i, j = int(w.big_rows[0]), int(w.big_cols[0])
        vals.append(C[i, j])
        bg.append(np.delete(C.ravel(), i * n + j).std())
    # c = rho |a|^2 + sqrt(1 - rho^2) <a, b~>: mean rho, sd about sqrt(2 rho^2 + 1 - rho^2) / sqrt(n)
    assert abs(np.mean(vals) - 0.8) < 4 * math.sqrt(1.64 / n) / math.sqrt(6)
    # background entries have variance 1 / n
    assert np.all(np.abs(np.array(bg) * math.sqrt(n) - 1.0) < 0.02)


def test_lightbulb_planted_pair_exact():
    for n in (256, 1024):
        w = I.lightbulb(n, 5)
        A, B = _np(w.A), _np(w.B)
        i, j = int(w.big_rows[0]), int(w.big_cols[0])
        flips = round(n * 0.2 / 2)
        assert abs((A[i] @ B[:, j]) - (1 - 2 * flips / n)) <= 1e-12
        assert np.all(np.abs(np.abs(A) * math.sqrt(n) - 1) < 1e-12)
        # column j* is row i* with exactly `flips` entries negated
        assert np.count_nonzero(A[i] != B[:, j]) == flips


def test_params_formula():
    # Section 5.6: d is the odd number 2 floor(c_d log2 n / 2) + 1
    assert I.params(1024, 1.0, 8)[0] == 11 and I.params(1024, 0.5, 8)[0] == 5
    assert I.params(4096, 0.75, 16) == (9, 16)
    assert all(I.params(n, c, 4)[0] % 2 == 1 for n in (64, 1024) for c in (0.3, 0.7, 1.3))


def test_correctness_counts_hand_case():
    C = np.array([[1.0, 0.0], [0.0, 0.3]])
    C_hat = np.array([[0.95, 0.6], [-0.05, 0.3]])
    # big (0,0): |0.95| >= 0.5, |0.95 - 1| <= 0.1; small: 0.6 is above 0.5 and
    # 0.6 away, -0.05 and 0.3 are below 0.5 and within 0.1
    assert O.correctness_counts(C_hat, C, [0], [0]).tolist() == [1, 2, 1, 2]
    # the comparisons are inclusive at both bounds; NaN satisfies none
    # (dyadic values, so every difference is exact)
    C2 = np.array([[1.0, 0.0], [0.0, 0.25]])
    C_hat2 = np.array([[0.5, 0.5], [np.nan, 0.375]])
    assert O.correctness_counts(C_hat2, C2, [0], [0], 0.5, 0.125).tolist() == [1, 2, 0, 1]
    assert O.correctness_counts(C_hat2, C2, [0], [0], 0.5, 0.5).tolist() == [1, 2, 1, 2]


def test_correctness_counts_invariants():
    rng = np.random.default_rng(2)
    C = rng.standard_normal((40, 30))
    big_r, big_c = np.array([0, 5, 39]), np.array([0, 29, 3])
    n_big, n_small = 3, 40 * 30 - 3
    got = O.correctness_counts(C, C, big_r, big_c, 0.0, 0.0)
    # exact estimates: every entry within any tolerance; |c| >= 0 for the big
    assert got.tolist() == [n_big, 0, n_big, n_small]
    far = C + 10.0
    got = O.correctness_counts(far, C, big_r, big_c, 100.0, 0.1)
    assert got.tolist() == [0, n_small, 0, 0]


def test_extract_reps_matches_decompress():
    w = small_random(60, 30, 50, 9, 5, seed=1)
    t1, t2 = O.hash_tables(w.keys, 60, 50, 9)
    p = O.bucket_sums(O.product(w.A, w.B), t1, t2, 9)
    rows = np.array([0, 59, 7, -1, 60, 3])
    cols = np.array([0, 49, 8, 2, 2, 50])
    x = O.extract_reps(p, t1, t2, rows, cols)
    ok = np.array([True, True, True, False, False, False])
    assert np.all(np.isnan(x[:, ~ok]))
    g = O.gather_reps(p, t1, t2, rows[ok], cols[ok])   # [d][r][c]
    for q in range(3):
        assert np.array_equal(x[:, q], g[:, q, q])
    assert np.array_equal(np.median(x[:, ok], axis=0),
                          O.extract_entries(p, t1, t2, rows[ok], cols[ok]))


def test_single_repetition_variance_bound_logunit():
    # Section 5.3 / Pagh's Theorem 3.1 on a LOGUNIT instance, d = 1 per draw:
    # the estimates of a big entry are unbiased with variance <= ||C||_F^2 / b
    n, log2b, draws = 64, 7, 1500
    w = I.logunit(n, 2)
    C = _np(w.A) @ _np(w.B)
    i, j = int(w.big_rows[0]), int(w.big_cols[0])
    keys = draw_keys(draws, 4040)
    t1, t2 = O.hash_tables(keys, n, n, log2b)
    p = O.bucket_sums(C, t1, t2, log2b)
    x = O.extract_reps(p, t1, t2, [i], [j])[:, 0]
    bound = (np.linalg.norm(C) ** 2 - C[i, j] ** 2) / (1 << log2b)
    assert abs(x.mean() - C[i, j]) <= 4 * math.sqrt(bound / draws)
    assert x.var() <= 1.3 * bound
