"""Seeded synthetic inputs for compressed matrix multiplication (FWHT form).

This module is shared by the oracle side (tests, CPU baseline) and the GPU
side (tests, bench) as the single source of inputs.  It holds none of the
method's arithmetic: no hashing, sketching, transforms or estimators.  Random
hash keys are drawn here and handed to both sides as plain 64-bit integers.

Recipes (Section 5.2 uses synthetic data only; the shapes below are the
planted-sparse workloads this implementation is measured on):

* ``hadamard_sparse``  A = D H Pi, B = Pi^T H^T X, so that C = A B = n D X is
  exactly sparse with ``nnz`` nonzeros (X has N(0,1) values at distinct
  uniformly random positions).
* ``planted_pm1``      A, B i.i.d. +-1; for each planted pair (i, j) row i of A
  is overwritten by ``scale`` times column j of B, so C[i, j] = scale * n.
* ``planted_pm1_two``  two planted columns per row of A (16384 pairs at
  n = 8192 need two per row): A[i] = scale * (B[:, j1] + B[:, j2]).
* ``gaussian_planted`` A, B i.i.d. N(0,1) with planted rows A[i] = scale*B[:, j].

Keys follow splitmix64 (Steele, Lea, Flood, OOPSLA 2014) seeded per
workload; per repetition t the pairs (a, c) are drawn in the order
h1, h2, s1, s2 (Section 4.2 draws two random 64-bit words per function).
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64_stream(seed: int, count: int) -> list[int]:
    """``count`` outputs of splitmix64 started from state ``seed``."""
    out = []
    state = seed & MASK64
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        out.append(z ^ (z >> 31))
    return out


def draw_keys(d: int, key_seed: int) -> np.ndarray:
    """Hash keys as uint64[d][4][2]: (a, c) for h1, h2, s1, s2 per repetition."""
    words = splitmix64_stream(key_seed, d * 8)
    return np.array(words, dtype=np.uint64).reshape(d, 4, 2)


def splitmix64_array(seed: int, count: int) -> np.ndarray:
    """splitmix64_stream as a uint64 array, computed without a Python loop:
    output i mixes the state seed + (i + 1) * 0x9E3779B97F4A7C15 (mod 2^64)."""
    i = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + i * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def draw_tabulation_keys(d: int, key_seed: int) -> np.ndarray:
    """Simple-tabulation tables as uint64[d][4][4][256]: per repetition, for
    h1, h2, s1, s2, four tables of 256 random words (one per key byte)."""
    return splitmix64_array(key_seed, d * 4 * 4 * 256).reshape(d, 4, 4, 256)


def draw_family_keys(family: str, d: int, key_seed: int) -> np.ndarray:
    """Keys for a hash family: uint64[d][4][2] for the multiply families,
    uint64[d][4][4][256] for simple tabulation."""
    if family in ("multiply_add_shift", "multiply_shift"):
        return draw_keys(d, key_seed)
    if family == "tabulation":
        return draw_tabulation_keys(d, key_seed)
    raise ValueError(f"unknown hash family {family!r}")


def sylvester(n: int) -> np.ndarray:
    """Sylvester-ordered +-1 Hadamard matrix of order n (power of two).

    Used only to build inputs with an exactly known sparse product."""
    h = np.ones((1, 1), dtype=np.float64)
    while h.shape[0] < n:
        h = np.block([[h, h], [h, -h]])
    return h


def hadamard_sparse(n: int, nnz: int, rng: np.random.Generator):
    """A = D H Pi, B = Pi^T H^T X; returns (A, B, C_exact) with C = n D X."""
    H = sylvester(n)
    dsign = rng.choice(np.array([-1.0, 1.0]), size=n)
    perm = rng.permutation(n)
    pos = rng.choice(n * n, size=nnz, replace=False)
    vals = rng.standard_normal(nnz)
    X = np.zeros((n, n))
    X.flat[pos] = vals
    DH = dsign[:, None] * H
    A = np.ascontiguousarray(DH[:, perm])
    B = np.ascontiguousarray((H.T @ X)[perm, :])
    C_exact = n * dsign[:, None] * X
    return A, B, C_exact


def _pm1(rng, shape):
    return (rng.integers(0, 2, size=shape, dtype=np.int8) * 2 - 1).astype(np.float64)


def planted_pm1(n: int, n_pairs: int, scale: float, rng: np.random.Generator,
                all_rows: bool = True):
    """+-1 matrices with ``n_pairs`` planted pairs (distinct rows i).

    Rows are a random permutation prefix; columns are drawn with replacement.
    Returns (A, B, rows, cols)."""
    A = _pm1(rng, (n, n))
    B = _pm1(rng, (n, n))
    if all_rows:
        rows = rng.permutation(n)[:n_pairs]
    else:
        rows = rng.choice(n, size=n_pairs, replace=False)
    cols = rng.integers(0, n, size=n_pairs)
    A[rows, :] = scale * B[:, cols].T
    return A, B, rows.astype(np.int64), cols.astype(np.int64)


def planted_pm1_two(n: int, scale: float, rng: np.random.Generator):
    """Two planted columns per row: A[i] = scale * (B[:, j1] + B[:, j2])."""
    A = _pm1(rng, (n, n))
    B = _pm1(rng, (n, n))
    j1 = rng.integers(0, n, size=n)
    j2 = (j1 + rng.integers(1, n, size=n)) % n
    A[:, :] = scale * (B[:, j1] + B[:, j2]).T
    rows = np.concatenate([np.arange(n), np.arange(n)])
    cols = np.concatenate([j1, j2])
    return A, B, rows.astype(np.int64), cols.astype(np.int64)


def gaussian_planted(n: int, n_pairs: int, scale: float, rng: np.random.Generator):
    """N(0,1) matrices with planted rows A[i] = scale * B[:, j] (all rows)."""
    A = rng.standard_normal((n, n))
    B = rng.standard_normal((n, n))
    rows = rng.permutation(n)[:n_pairs]
    cols = rng.integers(0, n, size=n_pairs)
    A[rows, :] = scale * B[:, cols].T
    return A, B, rows.astype(np.int64), cols.astype(np.int64)


class Workload(SimpleNamespace):
    """One (A, B, keys, log2b, d) problem plus its description fields."""

    def get(self, name, default=None):
        return getattr(self, name, default)


def exact_sparse_256(seed: int = 0) -> Workload:
    """n=256, b=2^12, d=5, float64, Hadamard-built, C exactly 256-sparse."""
    n, log2b, d = 256, 12, 5
    rng = np.random.default_rng(seed)
    A, B, C_exact = hadamard_sparse(n, 256, rng)
    return Workload(name="hadamard-sparse n=256 b=2^12 d=5 f64", n=n, log2b=log2b, d=d,
                    A=A, B=B, C_exact=C_exact, keys=draw_keys(d, 1000 + seed),
                    estimator="median", kind="exact")


def planted_4096(seed: int = 0) -> Workload:
    """n=4096, b=2^16, d=9, float64, +-1 with 4096 planted pairs at 4n."""
    n, log2b, d = 4096, 16, 9
    rng = np.random.default_rng(seed)
    A, B, rows, cols = planted_pm1(n, n, 4.0, rng)
    return Workload(name="planted-pm1 n=4096 b=2^16 d=9 f64", n=n, log2b=log2b, d=d,
                    A=A, B=B, rows=rows, cols=cols, tau=2.0 * n,
                    keys=draw_keys(d, 1000 + seed), estimator="median", kind="planted")


def planted_8192(seed: int = 0, gaussian: bool = False) -> Workload:
    """n=8192, b=2^18, d=9: 16384 planted pairs, two per row of A.

    ``gaussian=True`` gives the same shape with N(0,1) entries (planted
    scale 3, one pair per row) so that low-precision rounding is visible."""
    n, log2b, d = 8192, 18, 9
    rng = np.random.default_rng(seed)
    if gaussian:
        A, B, rows, cols = gaussian_planted(n, n, 3.0, rng)
        tau = 1.5 * n
    else:
        A, B, rows, cols = planted_pm1_two(n, 4.0, rng)
        tau = 2.0 * n
    return Workload(name=f"planted-{'gauss' if gaussian else 'pm1'} n=8192 b=2^18 d=9",
                    n=n, log2b=log2b, d=d, A=A, B=B, rows=rows, cols=cols, tau=tau,
                    keys=draw_keys(d, 1000 + seed), estimator="median", kind="planted")


def batched_mix(seed: int = 0, count: int = 64, sizes=(512, 1024, 2048, 4096)):
    """``count`` independent pairs, n uniform over ``sizes``, b=16n, d=7.

    The first half is Hadamard-built exactly sparse (nnz = n); the second
    half is +-1 with n/2 planted pairs (distinct rows) at 4n."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.array(sizes), size=count)
    out = []
    for p in range(count):
        n = int(ns[p])
        log2b = int(np.log2(16 * n))
        keys = draw_keys(7, 1000 + seed * count + p)
        if p < count // 2:
            A, B, C_exact = hadamard_sparse(n, n, rng)
            out.append(Workload(name=f"pair{p} hadamard n={n}", n=n, log2b=log2b, d=7,
                                A=A, B=B, C_exact=C_exact, keys=keys,
                                estimator="median", kind="exact"))
        else:
            A, B, rows, cols = planted_pm1(n, n // 2, 4.0, rng, all_rows=False)
            out.append(Workload(name=f"pair{p} planted n={n}", n=n, log2b=log2b, d=7,
                                A=A, B=B, rows=rows, cols=cols, tau=2.0 * n, keys=keys,
                                estimator="median", kind="planted"))
    return out


def gradient_2048(seed: int = 0) -> Workload:
    """n=2048, b=2^15, d=7, mean estimator; N(0,1) with 2048 planted rows
    A[i] = 3 B[:, j]; upstream weight W ~ N(0,1)."""
    n, log2b, d = 2048, 15, 7
    rng = np.random.default_rng(seed)
    A, B, rows, cols = gaussian_planted(n, n, 3.0, rng)
    W = rng.standard_normal((n, n))
    return Workload(name="gaussian-planted n=2048 b=2^15 d=7 mean", n=n, log2b=log2b, d=d,
                    A=A, B=B, W=W, rows=rows, cols=cols, keys=draw_keys(d, 1000 + seed),
                    estimator="mean", kind="planted")


def small_random(n_rows: int, n_inner: int, n_cols: int, log2b: int, d: int, seed: int,
                 integer: bool = False) -> Workload:
    """Small dense problem for parity sweeps (ragged shapes allowed)."""
    rng = np.random.default_rng(seed)
    if integer:
        A = rng.integers(-3, 4, size=(n_rows, n_inner)).astype(np.float64)
        B = rng.integers(-3, 4, size=(n_inner, n_cols)).astype(np.float64)
    else:
        A = rng.standard_normal((n_rows, n_inner))
        B = rng.standard_normal((n_inner, n_cols))
    return Workload(name=f"random {n_rows}x{n_inner}x{n_cols} b=2^{log2b} d={d}",
                    n=n_inner, n_rows=n_rows, n_cols=n_cols, log2b=log2b, d=d, A=A, B=B,
                    keys=draw_keys(d, 7000 + seed), estimator="median", kind="random")
