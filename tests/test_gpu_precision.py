"""Precision form (bf16 / fp16 operands on MFMA, float32 accumulation,
float64 cross-k sum and inverse) against the float64 oracle (GPU).

Element by element throughout.  Where every rounded quantity is an integer
the low precision represents exactly, the form is exact and p must equal the
oracle's bucket sums bit for bit (one slice and 2 to 16 slices, collision
chains merged ahead of the kernel and not).  On real data every entry of p
and C_hat is held to the tolerance derived in tests/numerics.py from the
rounding points of the form: the operand copies, the collision sums, the
results of matrix passes 1 to 3 (each rounded to the low precision), the
float32 sums inside the matrix instructions and the float32 accumulation
over 64 values of k between float64 flushes."""
import numpy as np
import pytest

import oracle as O
import paper_2601_09477_amd as cmm
from workloads import draw_keys, planted_8192, small_random
from tests.gpu_util import announce, dev, host, torch
from tests.numerics import U_BF16, U_F16, p_tolerance, round_bf16, round_f16

K_FLUSH = 128    # values of k summed in float32 between float64 flushes
LEVELS_LP = 4    # low-precision roundings after the operand copy: collision sums, passes 1-3
LEVELS_32 = 16   # float32 roundings inside the matrix passes (4 passes of 16-term sums)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch().cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()


def _ref(w, n_rows, n_cols):
    t1, t2 = O.hash_tables(w.keys, n_rows, n_cols, w.log2b)
    C = O.product(w.A, w.B)
    return C, O.bucket_sums(C, t1, t2, w.log2b), t1, t2


@pytest.mark.parametrize("compute", ["f16", "bf16"])
def test_mfma_small_integers_exact(compute):
    # Entries in {-1, 0, 1} with 200 inner rows: every sketch value and
    # every transform intermediate is an integer of magnitude <= 200 * 16 <
    # 2^12 before the final float32 passes ... bf16 keeps 8 significant bits,
    # so it is exact only while |values| <= 256: use 32 inner rows for bf16.
    n_inner = 200 if compute == "f16" else 32
    announce(f"mfma {compute} small integers n_inner={n_inner}")
    rng = np.random.default_rng(21)
    A = rng.integers(-1, 2, size=(300, n_inner)).astype(np.float64)
    B = rng.integers(-1, 2, size=(n_inner, 260)).astype(np.float64)
    keys = draw_keys(3, 77)
    from types import SimpleNamespace
    w = SimpleNamespace(A=A, B=B, keys=keys, log2b=14, d=3)
    res = cmm.estimate(dev(A), dev(B), 3, 14, keys=keys, compute=compute)
    C, p_ref, t1, t2 = _ref(w, 300, 260)
    assert np.array_equal(host(res.p), p_ref)
    assert np.array_equal(host(res.C_hat), O.extract(p_ref, t1, t2, "median"))


def _rounder(compute):
    return (round_bf16, U_BF16) if compute == "bf16" else (round_f16, U_F16)


def _sparse_pm1(rng, n_lines, length, per_line):
    """+-1 entries, exactly `per_line` nonzeros in each of `n_lines` lines."""
    M = np.zeros((n_lines, length))
    for r in range(n_lines):
        idx = rng.choice(length, size=per_line, replace=False)
        M[r, idx] = rng.integers(0, 2, size=per_line) * 2.0 - 1.0
    return M


def _exact_operands(n_rows, n_inner, n_cols, compute, seed):
    # Column k of A and row k of B have `per` entries +-1: every sketch
    # value, collision sum and partial transform is an integer of magnitude
    # <= per (exact in bf16 for per <= 256, in fp16 for per <= 2048), every
    # product |X_u Y_u| <= per^2 and a float32 run of K_FLUSH such products
    # stays below 2^24, so the form computes p exactly.
    per = 192 if compute == "bf16" else 360
    rng = np.random.default_rng(seed)
    A = np.ascontiguousarray(_sparse_pm1(rng, n_inner, n_rows, per).T)
    B = _sparse_pm1(rng, n_inner, n_cols, per)
    assert per * per * K_FLUSH < 2 ** 24
    return A, B


def _sparse_reference(A, B, t1, t2, log2b):
    import scipy.sparse as sp
    C = (sp.csr_matrix(A) @ sp.csr_matrix(B)).tocoo()
    return O.bucket_sums_sparse(C.row, C.col, C.data, t1, t2, log2b)


@pytest.mark.parametrize("log2b", [15, 16, 17, 18])
@pytest.mark.parametrize("compute", ["bf16", "f16"])
def test_mfma_multislice_exact(compute, log2b):
    # b = 2^15 .. 2^18: 2 to 16 slices of 2^14 with the folded signs of the
    # top bits; 4096 rows into 2^14 buckets give collision chains, the two-row
    # ones merged ahead of the kernel.  Bit-exact, element by element.
    n, n_inner, d = 4096, 96, 3
    announce(f"mfma {compute} multi-slice exact log2b={log2b}")
    A, B = _exact_operands(n, n_inner, n, compute, 100 + log2b)
    keys = draw_keys(d, 300 + log2b)
    res = cmm.estimate(dev(A), dev(B), d, log2b, keys=keys, compute=compute)
    t1, t2 = O.hash_tables(keys, n, n, log2b)
    p_ref = _sparse_reference(A, B, t1, t2, log2b)
    p = host(res.p)
    assert np.array_equal(p, p_ref), np.max(np.abs(p - p_ref))
    rows = np.arange(0, n, 37)
    assert np.array_equal(host(res.C_hat)[rows], O.extract(p_ref, t1, t2, "median", rows=rows))


@pytest.mark.parametrize("compute", ["bf16", "f16"])
def test_mfma_multislice_exact_unmerged(compute):
    # n = 12000: the chains left to descriptors exceed their slots, so no
    # chain is merged ahead of the kernel and the fix-ups take every chain.
    n, n_inner, d, log2b = 12000, 64, 3, 15
    announce(f"mfma {compute} multi-slice exact unmerged n={n}")
    A, B = _exact_operands(n, n_inner, n, compute, 7)
    keys = draw_keys(d, 99)
    res = cmm.estimate(dev(A), dev(B), d, log2b, keys=keys, compute=compute)
    t1, t2 = O.hash_tables(keys, n, n, log2b)
    p_ref = _sparse_reference(A, B, t1, t2, log2b)
    assert np.array_equal(host(res.p), p_ref)


@pytest.mark.parametrize("log2b", [14, 15, 16, 17, 18])
@pytest.mark.parametrize("compute", ["bf16", "f16"])
def test_mfma_gaussian_elementwise(compute, log2b):
    # Real data, every entry of p and of C_hat against the oracle: (1) on the
    # operands as the form rounds them (the oracle's bucket sums of the exact
    # product of the rounded copies), within the tolerance of the form's own
    # rounding points; (2) on the original operands, one rounding level more.
    announce(f"mfma {compute} gaussian elementwise log2b={log2b}")
    w = small_random(512, 96, 480, log2b, 3, seed=31 + log2b)
    rnd, u = _rounder(compute)
    res = cmm.estimate(dev(w.A), dev(w.B), w.d, w.log2b, keys=w.keys, compute=compute)
    p, C_hat = host(res.p), host(res.C_hat)
    t1, t2 = O.hash_tables(w.keys, 512, 480, w.log2b)
    for rounded in (True, False):
        A = rnd(w.A) if rounded else w.A
        B = rnd(w.B) if rounded else w.B
        p_ref = O.bucket_sums(O.product(A, B), t1, t2, w.log2b)
        tol = p_tolerance(A, B, w.log2b, u, LEVELS_LP + (0 if rounded else 1), K_FLUSH,
                          extra32=LEVELS_32)
        dp = np.abs(p - p_ref).max()
        dC = np.abs(C_hat - O.extract(p_ref, t1, t2, "median")).max()
        print(f"{compute} log2b={log2b} rounded={rounded}: max|dp| = {dp:.3e} "
              f"({dp / tol:.3f} of tol), max|dC| = {dC:.3e}", flush=True)
        assert dp <= tol and dC <= tol


def test_mfma_planted_8192_full_size():
    # The precision-form workload (n = 8192, b = 2^18, d = 9, +-1 with two
    # planted columns per row at 4n): p against the oracle's bucket sums of
    # the exact product, the error at the level measured for this workload
    # (bf16 8.1e-7 of max|p|, fp16 0), and on every 64th row the set of
    # estimates at or above tau = 2n equal to the oracle's (entries within the
    # largest deviation of tau excepted).
    from workloads.metrics import planted_recall
    announce("mfma planted n=8192 b=2^18 d=9 bf16 + f16 + f64")
    w = planted_8192(0)
    A, B = dev(w.A), dev(w.B)
    t1, t2 = O.hash_tables(w.keys, w.n, w.n, w.log2b)
    p_ref = O.bucket_sums(O.product(w.A, w.B), t1, t2, w.log2b)
    rows = np.arange(0, w.n, 64)
    C_ref_rows = O.extract(p_ref, t1, t2, "median", rows=rows)
    limit = {"f64": 0.0, "f16": 1e-6, "bf16": 4e-6}
    for compute in ("f64", "f16", "bf16"):
        res = cmm.estimate(A, B, w.d, w.log2b, keys=w.keys, compute=compute)
        p = host(res.p)
        C_hat = host(res.C_hat)
        dp = np.max(np.abs(p - p_ref))
        rel = dp / np.max(np.abs(p_ref))
        rec = planted_recall(C_hat, w.rows, w.cols, w.tau)
        print(f"{compute}: max|dp|/max|p| = {rel:.3e}, recall {rec['recalled']}/{rec['planted']}",
              flush=True)
        assert rel <= limit[compute]
        if compute == "f64":
            # integer data below 2^53: exact
            assert np.array_equal(p, p_ref)
            assert np.array_equal(C_hat[rows], C_ref_rows)
        clear = np.abs(np.abs(C_ref_rows) - w.tau) > dp
        assert np.array_equal((np.abs(C_hat[rows]) >= w.tau)[clear],
                              (np.abs(C_ref_rows) >= w.tau)[clear])
        assert rec["recall"] >= 1.0 - 2.0 / rec["planted"]
        del res, C_hat
        torch().cuda.empty_cache()


def test_mfma_gaussian_8192_against_oracle():
    # The N(0,1) variant of the same shape (one planted row per row of A at
    # scale 3): every entry of p against the oracle's bucket sums of the
    # exact float64 product, within the derived tolerance (operand copies
    # counted as a rounding level), C_hat on every 64th row likewise, and
    # every planted pair recalled.
    from workloads.metrics import planted_recall
    announce("mfma gaussian n=8192 b=2^18 d=9 bf16 + f16 against the oracle")
    w = planted_8192(0, gaussian=True)
    A, B = dev(w.A), dev(w.B)
    t1, t2 = O.hash_tables(w.keys, w.n, w.n, w.log2b)
    p_ref = O.bucket_sums(O.product(w.A, w.B), t1, t2, w.log2b)
    rows = np.arange(0, w.n, 64)
    C_ref_rows = O.extract(p_ref, t1, t2, "median", rows=rows)
    for compute in ("f16", "bf16"):
        u = U_BF16 if compute == "bf16" else U_F16
        tol = p_tolerance(w.A, w.B, w.log2b, u, LEVELS_LP + 1, K_FLUSH, extra32=LEVELS_32)
        res = cmm.estimate(A, B, w.d, w.log2b, keys=w.keys, compute=compute)
        p = host(res.p)
        C_hat = host(res.C_hat)
        dp = np.abs(p - p_ref).max()
        dC = np.abs(C_hat[rows] - C_ref_rows).max()
        rec = planted_recall(C_hat, w.rows, w.cols, w.tau)
        print(f"{compute}: max|dp| = {dp:.3e} ({dp / tol:.3f} of tol), rms(dp)/rms(p) = "
              f"{np.sqrt(np.mean((p - p_ref) ** 2) / np.mean(p_ref ** 2)):.3e}, "
              f"max|dC| = {dC:.3e}, recall {rec['recalled']}/{rec['planted']}", flush=True)
        assert dp <= tol and dC <= tol
        assert rec["recalled"] == rec["planted"]
        del res, C_hat
        torch().cuda.empty_cache()


@pytest.mark.parametrize("n,key_seed", [(10000, 10005), (10500, 10501), (12000, 12005)])
@pytest.mark.parametrize("compute", ["f16", "bf16"])
def test_mfma_merged_chains_overflow(n, key_seed, compute):
    # Per repetition and operand (counted from the oracle's tables): at
    # n = 10000 one operand's two-row chains are merged and its chains of
    # three or more rows take collision descriptors; at n = 10500 the
    # two-row chains outnumber the sums the kernel can stage beside a row,
    # so the rest take descriptors; at n = 12000 (and in one operand of each
    # of the others) the chains left to descriptors exceed their slots, so
    # none is merged ahead of the kernel.  Every entry of p against the
    # oracle on the rounded operands, within the derived tolerance.
    announce(f"mfma {compute} merged-chain overflow n={n}")
    rng = np.random.default_rng(n)
    n_inner, log2b, d = 16, 14, 3
    A = rng.standard_normal((n, n_inner))
    B = rng.standard_normal((n_inner, n))
    keys = draw_keys(d, key_seed)
    rnd, u = _rounder(compute)
    res = cmm.estimate(dev(A), dev(B), d, log2b, keys=keys, compute=compute)
    Ar, Br = rnd(A), rnd(B)
    t1, t2 = O.hash_tables(keys, n, n, log2b)
    p_ref = O.bucket_sums(O.product(Ar, Br), t1, t2, log2b)
    tol = p_tolerance(Ar, Br, log2b, u, LEVELS_LP, K_FLUSH, extra32=LEVELS_32)
    dp = np.abs(host(res.p) - p_ref).max()
    print(f"{compute} n={n}: max|dp| = {dp:.3e} ({dp / tol:.3f} of tol)", flush=True)
    assert dp <= tol
