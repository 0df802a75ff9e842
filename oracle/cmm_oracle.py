"""Oracle: the plain definitions behind Algorithm 1 (Compress / Decompress).

TEST INFRASTRUCTURE ONLY -- see the package docstring.  float64 throughout.

Conventions (readings of the paper where it is silent or inconsistent):
* indices are 0-based; h1/s1 hash the row index i of A, h2/s2 the column
  index j of B (Section 3.1);
* a hash table entry is a uint32 holding the bucket in bits [0, log2b) and
  the sign in bit 31 (1 means -1);
* the transform is the unnormalised Walsh-Hadamard transform in natural
  (Sylvester) order, H[u, r] = (-1)^popcount(u & r), so H H = b I; the
  inverse transform of Algorithm 1 is applied with the exact scale 2^-log2b,
  which makes p the XOR convolution of eq. (fwhtxorconvolution) exactly;
* the median needs an odd number of repetitions d (the formula for d in
  Section 5.6 always gives an odd number).
"""
from __future__ import annotations

import numpy as np

SIGN_BIT = np.uint32(1 << 31)


# --------------------------------------------------------------------- hashing
def multiply_add_shift(a: int, c: int, x: np.ndarray, out_bits: int) -> np.ndarray:
    """Section 4.2: h_{a,c}(x) = floor(((a x + c) mod 2^64) / 2^(64 - out_bits)).

    NumPy uint64 arithmetic wraps modulo 2^64, which is the "mod 2^64" of the
    64-bit multiplication and addition."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        v = np.uint64(a) * x + np.uint64(c)
    return (v >> np.uint64(64 - out_bits)).astype(np.uint64)


def hash_tables(keys: np.ndarray, n_rows: int, n_cols: int, log2b: int):
    """Algorithm 1, Compress (the draws of s1, s2, h1, h2 per repetition) with
    the Section 4.2 family; the sign hash is the same family with b = 2.

    keys: uint64 [d][4][2], rows (a, c) for h1, h2, s1, s2.
    Returns tab1 uint32[d][n_rows], tab2 uint32[d][n_cols]."""
    keys = np.asarray(keys, dtype=np.uint64)
    d = keys.shape[0]
    tab1 = np.zeros((d, n_rows), dtype=np.uint32)
    tab2 = np.zeros((d, n_cols), dtype=np.uint32)
    xr = np.arange(n_rows, dtype=np.uint64)
    xc = np.arange(n_cols, dtype=np.uint64)
    for t in range(d):
        (a1, c1), (a2, c2), (as1, cs1), (as2, cs2) = [(int(k[0]), int(k[1])) for k in keys[t]]
        h1 = multiply_add_shift(a1, c1, xr, log2b)
        h2 = multiply_add_shift(a2, c2, xc, log2b)
        s1 = multiply_add_shift(as1, cs1, xr, 1)   # 1 means sign -1
        s2 = multiply_add_shift(as2, cs2, xc, 1)
        tab1[t] = (h1 | (s1 << np.uint64(31))).astype(np.uint32)
        tab2[t] = (h2 | (s2 << np.uint64(31))).astype(np.uint32)
    return tab1, tab2


# Section 4.2 also names a simpler and a more complex family that the paper
# tried without reporting results.  Their definitions are not given there;
# the two below are the standard ones (readings, see the package docs).
def multiply_shift(a: int, x: np.ndarray, out_bits: int) -> np.ndarray:
    """The simpler family, read as multiply-shift (Dietzfelbinger, Hagerup,
    Katajainen, Penttonen 1997): the Section 4.2 family without the additive
    word, h_a(x) = floor(((a x) mod 2^64) / 2^(64 - out_bits)) with a odd
    (the low bit of the drawn word is set).  Universal, not 2-wise
    independent: x = 0 always lands in bucket 0 with sign +1."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        v = np.uint64(int(a) | 1) * x
    return (v >> np.uint64(64 - out_bits)).astype(np.uint64)


def tabulation(T: np.ndarray, x: np.ndarray, out_bits: int) -> np.ndarray:
    """The more complex family, simple tabulation (Patrascu and Thorup 2012):
    the 32-bit key x is cut into the bytes x_0 (least significant) .. x_3 and
    h(x) = T[0][x_0] xor T[1][x_1] xor T[2][x_2] xor T[3][x_3] over tables of
    random 64-bit words; the out_bits top bits of h(x) are the hash value."""
    x = np.asarray(x, dtype=np.uint64)
    T = np.asarray(T, dtype=np.uint64)
    v = np.zeros(x.shape, dtype=np.uint64)
    for q in range(4):
        v ^= T[q][((x >> np.uint64(8 * q)) & np.uint64(0xFF)).astype(np.int64)]
    return (v >> np.uint64(64 - out_bits)).astype(np.uint64)


def hash_tables_family(family: str, keys: np.ndarray, n_rows: int, n_cols: int, log2b: int):
    """hash_tables for a named family: "multiply_add_shift" (Section 4.2;
    keys uint64[d][4][2]), "multiply_shift" (keys uint64[d][4][2], the second
    word of each pair unused) or "tabulation" (keys uint64[d][4][4][256]: for
    h1, h2, s1, s2 the four byte tables).  Same table layout as hash_tables."""
    if family == "multiply_add_shift":
        return hash_tables(keys, n_rows, n_cols, log2b)
    keys = np.asarray(keys, dtype=np.uint64)
    d = keys.shape[0]
    xr = np.arange(n_rows, dtype=np.uint64)
    xc = np.arange(n_cols, dtype=np.uint64)
    tab1 = np.zeros((d, n_rows), dtype=np.uint32)
    tab2 = np.zeros((d, n_cols), dtype=np.uint32)
    for t in range(d):
        if family == "multiply_shift":
            f = [lambda x, bits, k=keys[t][q]: multiply_shift(int(k[0]), x, bits) for q in range(4)]
        elif family == "tabulation":
            f = [lambda x, bits, k=keys[t][q]: tabulation(k, x, bits) for q in range(4)]
        else:
            raise ValueError(f"unknown hash family {family!r}")
        h1, h2 = f[0](xr, log2b), f[1](xc, log2b)
        s1, s2 = f[2](xr, 1), f[3](xc, 1)
        tab1[t] = (h1 | (s1 << np.uint64(31))).astype(np.uint32)
        tab2[t] = (h2 | (s2 << np.uint64(31))).astype(np.uint32)
    return tab1, tab2


def bucket(tab: np.ndarray) -> np.ndarray:
    """Bucket index of a table entry."""
    return (np.asarray(tab) & np.uint32(0x7FFFFFFF)).astype(np.int64)


def sign(tab: np.ndarray) -> np.ndarray:
    """Sign (+1.0 / -1.0) of a table entry."""
    return np.where(np.asarray(tab) & SIGN_BIT, -1.0, 1.0)


# ------------------------------------------------------------------ sketching
def count_sketch(M: np.ndarray, tab: np.ndarray, side: int, k0: int, kc: int,
                 log2b: int) -> np.ndarray:
    """Algorithm 1, the two inner loops of Compress, for kc consecutive k.

    side 0 (A, n_rows x n_inner): out[t][kk][x] = sum_{i: h1(i)=x} s1(i) A[i, k0+kk]
    side 1 (B, n_inner x n_cols): out[t][kk][x] = sum_{j: h2(j)=x} s2(j) B[k0+kk, j]
    Rows (columns) are added in ascending index order."""
    d = tab.shape[0]
    b = 1 << log2b
    out = np.zeros((d, kc, b), dtype=np.float64)
    for t in range(d):
        h = bucket(tab[t])
        s = sign(tab[t])
        for idx in range(tab.shape[1]):
            vals = M[idx, k0:k0 + kc] if side == 0 else M[k0:k0 + kc, idx]
            out[t, :, h[idx]] += s[idx] * vals
    return out


# ------------------------------------------------------------------ transform
def wht(x: np.ndarray, scale: float = 1.0) -> np.ndarray:
    """Walsh-Hadamard transform along the last axis (Section 3.2): the
    textbook radix-2 butterflies (a, b) -> (a + b, a - b) over strides
    1, 2, 4, ..., giving natural order; then multiplied by ``scale``.
    Returns a new array."""
    y = np.array(x, dtype=np.float64, copy=True)
    b = y.shape[-1]
    assert b & (b - 1) == 0, "length must be a power of two"
    lead = y.shape[:-1]
    h = 1
    while h < b:
        v = y.reshape(lead + (b // (2 * h), 2, h))
        lo = v[..., 0, :].copy()
        hi = v[..., 1, :].copy()
        v[..., 0, :] = lo + hi
        v[..., 1, :] = lo - hi
        h *= 2
    if scale != 1.0:
        y *= scale
    return y


def wht_matrix(log2b: int) -> np.ndarray:
    """The definition H[u, r] = (-1)^popcount(u & r) (natural order)."""
    b = 1 << log2b
    u = np.arange(b, dtype=np.int64)
    and_ = u[:, None] & u[None, :]
    pop = np.zeros_like(and_)
    for bit in range(log2b):
        pop += (and_ >> bit) & 1
    return np.where(pop & 1, -1.0, 1.0)


def xor_convolution(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """eq. (fwhtxorconvolution): (x *xor y)[k] = sum_{i xor j = k} x[i] y[j]."""
    b = x.shape[-1]
    out = np.zeros(b)
    for i in range(b):
        for j in range(b):
            out[i ^ j] += x[i] * y[j]
    return out


# ----------------------------------------------------------------- accumulate
def accumulate(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Algorithm 1, p[t] += H{p_A} o H{p_B} summed over k (ascending):
    p_hat[t][u] = sum_kk X[t][kk][u] * Y[t][kk][u]."""
    d, kc, b = X.shape
    p_hat = np.zeros((d, b))
    for kk in range(kc):
        p_hat += X[:, kk, :] * Y[:, kk, :]
    return p_hat


# ------------------------------------------------------------------- compress
def compress_alg1(A: np.ndarray, B: np.ndarray, tab1: np.ndarray, tab2: np.ndarray,
                  log2b: int, k_chunk: int = 256) -> np.ndarray:
    """Algorithm 1, Compress, in the paper's order: per repetition, sketch
    column k of A and row k of B, transform both, add the pointwise product
    into p[t]; finally p[t] <- 2^-log2b H{p[t]}.  Returns p float64[d][b]."""
    d = tab1.shape[0]
    n_inner = A.shape[1]
    b = 1 << log2b
    p_hat = np.zeros((d, b))
    for k0 in range(0, n_inner, k_chunk):
        kc = min(k_chunk, n_inner - k0)
        X = wht(count_sketch(A, tab1, 0, k0, kc, log2b))
        Y = wht(count_sketch(B, tab2, 1, k0, kc, log2b))
        p_hat += accumulate(X, Y)
    return wht(p_hat, 2.0 ** -log2b)


def bucket_sums(C: np.ndarray, tab1: np.ndarray, tab2: np.ndarray, log2b: int,
                row_block: int = 512) -> np.ndarray:
    """The plain definition of the sketch p that Compress reaches (Section 3.2
    with eq. (fwhtxorconvolution), and the estimator decomposition of
    Section 6.4): p_t[x] = sum over (i, j) with h1(i) xor h2(j) = x of
    s1(i) s2(j) C[i, j].  Summed in row-major (i, j) order within blocks of
    ``row_block`` rows, blocks added in ascending order."""
    d = tab1.shape[0]
    b = 1 << log2b
    n_rows, n_cols = C.shape
    p = np.zeros((d, b))
    for t in range(d):
        h1, s1 = bucket(tab1[t]), sign(tab1[t])
        h2, s2 = bucket(tab2[t]), sign(tab2[t])
        for r0 in range(0, n_rows, row_block):
            r1 = min(n_rows, r0 + row_block)
            idx = (h1[r0:r1, None] ^ h2[None, :]).ravel()
            w = (s1[r0:r1, None] * s2[None, :] * C[r0:r1]).ravel()
            p[t] += np.bincount(idx, weights=w, minlength=b)
    return p


def bucket_sums_sparse(rows: np.ndarray, cols: np.ndarray, vals: np.ndarray, tab1: np.ndarray,
                       tab2: np.ndarray, log2b: int) -> np.ndarray:
    """The same definition as ``bucket_sums`` for a product C given by its
    nonzero entries C[rows[e], cols[e]] = vals[e] (zero entries add nothing):
    p_t[x] = sum over e with h1(rows[e]) xor h2(cols[e]) = x of
    s1(rows[e]) s2(cols[e]) vals[e]."""
    d = tab1.shape[0]
    b = 1 << log2b
    p = np.zeros((d, b))
    for t in range(d):
        idx = bucket(tab1[t][rows]) ^ bucket(tab2[t][cols])
        w = sign(tab1[t][rows]) * sign(tab2[t][cols]) * np.asarray(vals, dtype=np.float64)
        p[t] = np.bincount(idx, weights=w, minlength=b)
    return p


def product(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """C = A B in float64 (library matmul as a step)."""
    return np.asarray(A, dtype=np.float64) @ np.asarray(B, dtype=np.float64)


# -------------------------------------------------------------------- extract
def gather_reps(p: np.ndarray, tab1: np.ndarray, tab2: np.ndarray,
                rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Algorithm 1, Decompress: x_t = s1[t](i) s2[t](j) p[t][h1[t](i) xor h2[t](j)]
    for every (i, j) in rows x cols.  Returns float64[d][len(rows)][len(cols)]."""
    d = p.shape[0]
    out = np.empty((d, len(rows), len(cols)))
    for t in range(d):
        h1, s1 = bucket(tab1[t][rows]), sign(tab1[t][rows])
        h2, s2 = bucket(tab2[t][cols]), sign(tab2[t][cols])
        out[t] = s1[:, None] * s2[None, :] * p[t][h1[:, None] ^ h2[None, :]]
    return out


def extract(p: np.ndarray, tab1: np.ndarray, tab2: np.ndarray, estimator: str = "median",
            rows=None, cols=None, row_block: int = 256) -> np.ndarray:
    """Algorithm 1, Decompress, for a dense block of entries: Median(x) over
    the d repetitions (odd d), or the mean over d (the mean-over-d estimator;
    each repetition is unbiased, Section 3.1)."""
    d = p.shape[0]
    rows = np.arange(tab1.shape[1]) if rows is None else np.asarray(rows)
    cols = np.arange(tab2.shape[1]) if cols is None else np.asarray(cols)
    if estimator == "median" and d % 2 == 0:
        raise ValueError("median estimator needs an odd number of repetitions")
    out = np.empty((len(rows), len(cols)))
    for r0 in range(0, len(rows), row_block):
        x = gather_reps(p, tab1, tab2, rows[r0:r0 + row_block], cols)
        out[r0:r0 + row_block] = np.median(x, axis=0) if estimator == "median" else x.mean(axis=0)
    return out


def extract_topk(p: np.ndarray, tab1: np.ndarray, tab2: np.ndarray, k: int,
                 estimator: str = "median"):
    """The k entries of largest |C_hat| of Algorithm 1's Decompress over the
    whole block (the large entries of the product, Section 1): the dense
    estimate, then a plain sort by |C_hat| descending with ties broken by the
    smaller row-major index.  Returns (rows, cols, vals)."""
    C_hat = extract(p, tab1, tab2, estimator)
    n_cols = C_hat.shape[1]
    flat = C_hat.ravel()
    idx = np.arange(flat.size)
    order = np.lexsort((idx, -np.abs(flat)))[:k]
    return order // n_cols, order % n_cols, flat[order]


def extract_entries(p: np.ndarray, tab1: np.ndarray, tab2: np.ndarray, rows, cols,
                    estimator: str = "median") -> np.ndarray:
    """Algorithm 1, Decompress, at a list of entries (rows[q], cols[q]): the
    median (odd d) or mean over t of s1 s2 p[t][h1 xor h2]; NaN for an index
    outside the tables."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    d = p.shape[0]
    out = np.full(len(rows), np.nan)
    ok = (rows >= 0) & (rows < tab1.shape[1]) & (cols >= 0) & (cols < tab2.shape[1])
    r, c = rows[ok], cols[ok]
    x = np.empty((d, len(r)))
    for t in range(d):
        x[t] = sign(tab1[t][r]) * sign(tab2[t][c]) * p[t][bucket(tab1[t][r]) ^ bucket(tab2[t][c])]
    out[ok] = np.median(x, axis=0) if estimator == "median" else x.mean(axis=0)
    return out


# ------------------------------------------------ Pagh's FFT form (Section 3.1)
def cyclic_convolution(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Section 2: (x * y)[k] = sum over i + j = k (mod b) of x[i] y[j], by the
    definition (O(b^2); for checks on small b)."""
    b = len(x)
    out = np.zeros(b)
    for i in range(b):
        for j in range(b):
            out[(i + j) % b] += x[i] * y[j]
    return out


def compress_fft(A: np.ndarray, B: np.ndarray, tab1: np.ndarray, tab2: np.ndarray,
                 log2b: int, k_chunk: int = 256) -> np.ndarray:
    """Pagh's Compress (Section 3.1): per repetition, count-sketch column k
    of A and row k of B, take their discrete Fourier transforms, add the
    pointwise product; finally p[t] = inverse transform, which is the cyclic
    convolution p_A * p_B summed over k.  The transform is numpy.fft (a
    library step).  Returns p float64[d][b] (the real part)."""
    d = tab1.shape[0]
    n_inner = A.shape[1]
    b = 1 << log2b
    P = np.zeros((d, b), dtype=np.complex128)
    for k0 in range(0, n_inner, k_chunk):
        kc = min(k_chunk, n_inner - k0)
        X = np.fft.fft(count_sketch(A, tab1, 0, k0, kc, log2b), axis=-1)
        Y = np.fft.fft(count_sketch(B, tab2, 1, k0, kc, log2b), axis=-1)
        P += (X * Y).sum(axis=1)
    return np.fft.ifft(P, axis=-1).real


def bucket_sums_cyclic(C: np.ndarray, tab1: np.ndarray, tab2: np.ndarray, log2b: int,
                       row_block: int = 512) -> np.ndarray:
    """The plain definition Pagh's Compress reaches: p_t[x] = sum over
    (i, j) with h1(i) + h2(j) = x (mod b) of s1(i) s2(j) C[i, j]
    (Section 3.1: h(i, j) = h1(i) + h2(j) mod b, s(i, j) = s1(i) s2(j))."""
    d = tab1.shape[0]
    b = 1 << log2b
    n_rows = C.shape[0]
    p = np.zeros((d, b))
    for t in range(d):
        h1, s1 = bucket(tab1[t]), sign(tab1[t])
        h2, s2 = bucket(tab2[t]), sign(tab2[t])
        for r0 in range(0, n_rows, row_block):
            r1 = min(n_rows, r0 + row_block)
            idx = ((h1[r0:r1, None] + h2[None, :]) % b).ravel()
            w = (s1[r0:r1, None] * s2[None, :] * C[r0:r1]).ravel()
            p[t] += np.bincount(idx, weights=w, minlength=b)
    return p


def extract_cyclic(p: np.ndarray, tab1: np.ndarray, tab2: np.ndarray,
                   estimator: str = "median") -> np.ndarray:
    """Pagh's Decompress: Median_t s1_t(i) s2_t(j) p[t][(h1_t(i) + h2_t(j)) mod b]
    (or the mean) for every (i, j)."""
    d, b = p.shape
    if estimator == "median" and d % 2 == 0:
        raise ValueError("median estimator needs an odd number of repetitions")
    x = np.empty((d, tab1.shape[1], tab2.shape[1]))
    for t in range(d):
        h1, s1 = bucket(tab1[t]), sign(tab1[t])
        h2, s2 = bucket(tab2[t]), sign(tab2[t])
        x[t] = s1[:, None] * s2[None, :] * p[t][(h1[:, None] + h2[None, :]) % b]
    return np.median(x, axis=0) if estimator == "median" else x.mean(axis=0)


def extract_reps(p: np.ndarray, tab1: np.ndarray, tab2: np.ndarray, rows, cols) -> np.ndarray:
    """The d single-repetition values of Algorithm 1's Decompress at a list
    of entries, before the median: out[t][q] = s1_t s2_t p[t][h1_t xor h2_t]
    at (rows[q], cols[q]); NaN for an index outside the tables."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    d = p.shape[0]
    out = np.full((d, len(rows)), np.nan)
    ok = (rows >= 0) & (rows < tab1.shape[1]) & (cols >= 0) & (cols < tab2.shape[1])
    r, c = rows[ok], cols[ok]
    for t in range(d):
        out[t, ok] = sign(tab1[t][r]) * sign(tab2[t][c]) * p[t][bucket(tab1[t][r]) ^ bucket(tab2[t][c])]
    return out


def correctness_counts(C_hat: np.ndarray, C: np.ndarray, big_rows, big_cols,
                       threshold: float = 0.5, tolerance: float = 0.1) -> np.ndarray:
    """Section 5.4: with B the big entries and S all others,
    [#B with |c~| >= thr, #S with |c~| <= thr, #B with |c~ - c| <= tol,
     #S with |c~ - c| <= tol] as int64."""
    C_hat = np.asarray(C_hat, dtype=np.float64)
    big = np.zeros(C_hat.shape, dtype=bool)
    big[np.asarray(big_rows, dtype=np.int64), np.asarray(big_cols, dtype=np.int64)] = True
    small = ~big
    mag = np.abs(C_hat)
    err = np.abs(C_hat - C)
    with np.errstate(invalid="ignore"):
        return np.array([np.count_nonzero(big & (mag >= threshold)),
                         np.count_nonzero(small & (mag <= threshold)),
                         np.count_nonzero(big & (err <= tolerance)),
                         np.count_nonzero(small & (err <= tolerance))], dtype=np.int64)


def estimate(A: np.ndarray, B: np.ndarray, keys: np.ndarray, log2b: int,
             estimator: str = "median"):
    """Compress + dense Decompress through the plain definition.
    Returns (C_hat, p, tab1, tab2)."""
    tab1, tab2 = hash_tables(keys, A.shape[0], B.shape[1], log2b)
    p = bucket_sums(product(A, B), tab1, tab2, log2b)
    return extract(p, tab1, tab2, estimator), p, tab1, tab2


# ------------------------------------------------------------------- gradient
def grad_mean(A: np.ndarray, B: np.ndarray, W: np.ndarray, tab1: np.ndarray,
              tab2: np.ndarray, log2b: int):
    """Gradient of L = sum(W o C_hat) for the mean-over-d estimator.

    C_hat = (1/d) sum_t L_t(A B) with L_t(C)[i, j] = s1 s2 p_t[h1(i) xor h2(j)]
    and p_t the bucket sums of C.  L_t is self-adjoint (its kernel
    s(i,j) s(i',j') [h(i,j) = h(i',j')] is symmetric), so dL/dC = G =
    (1/d) sum_t L_t(W), and by the product rule dA = G B^T, dB = A^T G."""
    q = bucket_sums(W, tab1, tab2, log2b)
    G = extract(q, tab1, tab2, "mean")
    return G @ B.T, A.T @ G, G
