"""Parity of every C-ABI call with the oracle (GPU; run on an MI355X).

Integer-valued inputs keep every float64 intermediate below 2^53, so the
GPU and the oracle must agree bit for bit whatever the summation order;
real-valued inputs are compared with the tolerance 1e-9 * ||C||_F / n.
"""
import numpy as np
import pytest

import oracle as O
import paper_2601_09477_amd as cmm
from workloads import draw_keys, exact_sparse_256, hadamard_sparse, small_random
from tests.gpu_util import announce, dev, host, tables_dev, torch
from tests.numerics import f32_tolerance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    t = torch()
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()


# ---------------------------------------------------------------- hash
@pytest.mark.parametrize("d,n_rows,n_cols,log2b", [
    (1, 1, 1, 1), (3, 257, 100, 7), (9, 4096, 4096, 16), (5, 1000, 3, 30), (2, 70000, 5, 18)])
def test_hash_bit_exact(d, n_rows, n_cols, log2b):
    announce(f"hash d={d} n={n_rows}x{n_cols} log2b={log2b}")
    t = torch()
    keys = draw_keys(d, 31 * d + log2b)
    tab1 = t.empty((d, n_rows), dtype=t.int32, device="cuda")
    tab2 = t.empty((d, n_cols), dtype=t.int32, device="cuda")
    cmm.cmm_hash(cmm.keys_tensor(keys), d, n_rows, n_cols, log2b, tab1, tab2)
    r1, r2 = O.hash_tables(keys, n_rows, n_cols, log2b)
    assert np.array_equal(cmm.tables_to_numpy(tab1), r1)
    assert np.array_equal(cmm.tables_to_numpy(tab2), r2)


# --------------------------------------------------------------- sketch
@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("rows,cols,log2b,k0,kc", [
    (37, 19, 5, 0, 19), (300, 129, 14, 7, 100), (130, 260, 13, 250, 10), (64, 64, 3, 0, 64),
    # more hits per window than one hit list holds (segments), and one
    # window of two buckets (long rank chains)
    (5000, 40, 4, 3, 30), (3000, 9, 1, 0, 9)])
def test_sketch_f64_bit_exact(side, rows, cols, log2b, k0, kc):
    if side == 1:
        rows, cols = cols, rows   # B is n_inner x n_cols
    n_inner = cols if side == 0 else rows
    if k0 + kc > n_inner:
        k0 = max(0, n_inner - kc)
        kc = min(kc, n_inner)
    announce(f"sketch f64 side={side} {rows}x{cols} log2b={log2b} k0={k0} kc={kc}")
    t = torch()
    rng = np.random.default_rng(rows + cols + log2b)
    M = rng.standard_normal((rows, cols))          # real data: same order => bit exact
    d = 3
    n_idx = rows if side == 0 else cols
    tab = O.hash_tables(draw_keys(d, 5 + side), n_idx, n_idx, log2b)[side]
    out = t.empty((d, kc, 1 << log2b), dtype=t.float64, device="cuda")
    cmm.cmm_sketch(side, dev(M), rows, cols, cols, tables_dev(tab), d, log2b, k0, kc, out)
    want = O.count_sketch(M, tab, side, k0, kc, log2b)
    assert np.array_equal(host(out), want)


@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("rows,cols,log2b,k0,kc", [(300, 129, 14, 7, 100), (5000, 40, 4, 3, 30)])
def test_sketch_mixed_dtypes_bit_exact(side, rows, cols, log2b, k0, kc):
    # float32 input into float64 sketches (the values widen exactly and are
    # summed in float64 in ascending index order), and float64 input into
    # float32 sketches (summed in float64, rounded once)
    if side == 1:
        rows, cols = cols, rows
    n_inner = cols if side == 0 else rows
    if k0 + kc > n_inner:
        k0 = max(0, n_inner - kc)
        kc = min(kc, n_inner)
    announce(f"sketch mixed dtypes side={side} {rows}x{cols} log2b={log2b} k0={k0} kc={kc}")
    t = torch()
    rng = np.random.default_rng(rows + 3 * cols + log2b)
    M = rng.standard_normal((rows, cols))
    M32 = M.astype(np.float32)
    d = 3
    n_idx = rows if side == 0 else cols
    tab = O.hash_tables(draw_keys(d, 15 + side), n_idx, n_idx, log2b)[side]
    out64 = t.empty((d, kc, 1 << log2b), dtype=t.float64, device="cuda")
    cmm.cmm_sketch(side, dev(M32, t.float32), rows, cols, cols, tables_dev(tab), d, log2b, k0, kc,
                   out64)
    assert np.array_equal(host(out64), O.count_sketch(M32.astype(np.float64), tab, side, k0, kc,
                                                      log2b))
    out32 = t.empty((d, kc, 1 << log2b), dtype=t.float32, device="cuda")
    cmm.cmm_sketch(side, dev(M), rows, cols, cols, tables_dev(tab), d, log2b, k0, kc, out32)
    want = O.count_sketch(M, tab, side, k0, kc, log2b).astype(np.float32)
    assert np.array_equal(out32.cpu().numpy(), want)


def test_sketch_f32_close():
    announce("sketch f32")
    t = torch()
    rng = np.random.default_rng(1)
    M = rng.standard_normal((200, 50)).astype(np.float32)
    tab = O.hash_tables(draw_keys(2, 9), 200, 200, 9)[0]
    out = t.empty((2, 50, 512), dtype=t.float32, device="cuda")
    cmm.cmm_sketch(0, dev(M), 200, 50, 50, tables_dev(tab), 2, 9, 0, 50, out)
    want = O.count_sketch(M.astype(np.float64), tab, 0, 0, 50, 9)
    assert np.max(np.abs(host(out) - want)) <= 200 * 2.0 ** -23 * np.abs(M).max() * 2


# ----------------------------------------------------------------- fwht
@pytest.mark.parametrize("log2b,batch", [(1, 3), (4, 1), (7, 5), (12, 2), (13, 3), (14, 3),
                                         (15, 2), (16, 2), (17, 2), (18, 1), (20, 1)])
def test_fwht_integer_exact_and_inverse(log2b, batch):
    announce(f"fwht log2b={log2b} batch={batch}")
    rng = np.random.default_rng(log2b)
    x = rng.integers(-100, 100, size=(batch, 1 << log2b)).astype(np.float64)
    g = dev(x)
    cmm.cmm_fwht(g, batch, log2b, 1.0)
    assert np.array_equal(host(g), O.wht(x))
    cmm.cmm_fwht(g, batch, log2b, 2.0 ** -log2b)
    assert np.array_equal(host(g), x)


@pytest.mark.parametrize("log2b", [12, 13, 16])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fwht_unaligned_integer_exact(log2b, dtype):
    """Vectors starting one element past an aligned address (the pass stores
    elements one by one there), float64 and float32 (integer data: exact)."""
    announce(f"fwht unaligned log2b={log2b} {dtype}")
    t = torch()
    rng = np.random.default_rng(40 + log2b)
    batch = 3
    x = rng.integers(-100, 100, size=(batch, 1 << log2b))
    tdt = t.float64 if dtype == "f64" else t.float32
    buf = t.zeros(batch * (1 << log2b) + 1, dtype=tdt, device="cuda")
    g = buf[1:]
    g.copy_(t.from_numpy(x.reshape(-1)).to(tdt))
    cmm.cmm_fwht(g, batch, log2b, 1.0)
    assert np.array_equal(g.cpu().double().numpy().reshape(batch, -1), O.wht(x.astype(np.float64)))
    assert float(buf[0]) == 0.0
    cmm.cmm_fwht(g, batch, log2b, 2.0 ** -log2b)
    assert np.array_equal(g.cpu().double().numpy().reshape(batch, -1), x.astype(np.float64))


@pytest.mark.parametrize("log2b", [9, 16])
def test_fwht_real_close(log2b):
    announce(f"fwht real log2b={log2b}")
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 1 << log2b))
    for dt, tol in ((np.float64, 1e-13), (np.float32, 3e-6)):
        g = dev(x.astype(dt))
        cmm.cmm_fwht(g, 3, log2b, 1.0)
        want = O.wht(x)
        scale = np.sqrt(1 << log2b) * log2b
        assert np.max(np.abs(host(g) - want)) <= tol * scale


# ----------------------------------------------------------- accumulate
@pytest.mark.parametrize("log2b,kc,dtype,offset", [
    (10, 17, "f64", 0), (1, 9, "f64", 0), (12, 8, "f32", 0), (10, 17, "f64", 1),
    (11, 5, "f32", 1), (1, 9, "f32", 0), (2, 12, "f32", 0), (13, 3, "f64", 0)])
def test_accumulate_bit_exact(log2b, kc, dtype, offset):
    """Aligned operands and operands one element past an aligned address;
    tails of kc below the 8-wide load groups; float32 operands widen
    exactly; p_hat starts nonzero (the sums are added into it)."""
    announce(f"accumulate log2b={log2b} kc={kc} {dtype} offset={offset}")
    t = torch()
    rng = np.random.default_rng(3 + log2b)
    d, b = 3, 1 << log2b
    ndt = np.float64 if dtype == "f64" else np.float32
    X = rng.standard_normal((d, kc, b)).astype(ndt)
    Y = rng.standard_normal((d, kc, b)).astype(ndt)
    p0 = rng.standard_normal((d, b))
    tdt = t.float64 if dtype == "f64" else t.float32
    bx = t.zeros(d * kc * b + offset, dtype=tdt, device="cuda")
    by = t.zeros(d * kc * b + offset, dtype=tdt, device="cuda")
    bp = t.zeros(d * b + offset, dtype=t.float64, device="cuda")
    gx, gy, p = bx[offset:], by[offset:], bp[offset:]
    gx.copy_(t.from_numpy(X.reshape(-1)))
    gy.copy_(t.from_numpy(Y.reshape(-1)))
    p.copy_(t.from_numpy(p0.reshape(-1)))
    cmm.cmm_accumulate(gx, gy, d, kc, log2b, p)
    got = p.cpu().numpy().reshape(d, b)
    # the starting p_hat enters the oracle as a first term p0 * 1 (exact), so
    # the oracle's ascending sum is the same sequence of rounded adds
    Xd = np.concatenate([p0[:, None, :], X.astype(np.float64)], axis=1)
    Yd = np.concatenate([np.ones((d, 1, b)), Y.astype(np.float64)], axis=1)
    want = O.accumulate(Xd, Yd)
    diff = np.abs(got - want)
    print("accumulate max diff", diff.max(), "count", np.count_nonzero(diff), flush=True)
    assert np.array_equal(got, want)


# -------------------------------------------------------------- extract
@pytest.mark.parametrize("d", [1, 3, 5, 7, 9, 11, 13, 15, 17, 21, 23])
@pytest.mark.parametrize("estimator", ["median", "mean"])
def test_extract_bit_exact(d, estimator):
    announce(f"extract d={d} {estimator}")
    t = torch()
    rng = np.random.default_rng(d)
    log2b, n_rows, n_cols = 9, 37, 300
    p = rng.standard_normal((d, 1 << log2b))
    t1, t2 = O.hash_tables(draw_keys(d, 40 + d), n_rows, n_cols, log2b)
    C = t.empty((n_rows, n_cols), dtype=t.float64, device="cuda")
    est = cmm.CMM_MEDIAN if estimator == "median" else cmm.CMM_MEAN
    cmm.cmm_extract(dev(p), tables_dev(t1), tables_dev(t2), d, n_rows, n_cols, log2b, est, C)
    want = O.extract(p, t1, t2, estimator)
    if estimator == "median":
        assert np.array_equal(host(C), want)
    else:
        assert np.allclose(host(C), want, rtol=0, atol=1e-15 * np.abs(p).max() * d)


# ------------------------------------------------------------- estimate
def _estimate_and_compare(w, n_rows, n_cols, exact, compute="f64"):
    t = torch()
    A, B = w.A, w.B
    res = cmm.estimate(dev(A), dev(B), w.d, w.log2b, keys=w.keys, compute=compute,
                       estimator=w.get("estimator", "median"))
    t1, t2 = O.hash_tables(w.keys, n_rows, n_cols, w.log2b)
    assert np.array_equal(cmm.tables_to_numpy(res.tab1), t1)
    assert np.array_equal(cmm.tables_to_numpy(res.tab2), t2)
    C = O.product(A, B)
    p_ref = O.bucket_sums(C, t1, t2, w.log2b)
    C_ref = O.extract(p_ref, t1, t2, w.get("estimator", "median"))
    p_gpu, C_gpu = host(res.p), host(res.C_hat)
    tol = 1e-9 * np.linalg.norm(C) / max(1, A.shape[1])
    if exact:
        assert np.array_equal(p_gpu, p_ref)
        assert np.array_equal(C_gpu, C_ref)
    else:
        assert np.max(np.abs(p_gpu - p_ref)) <= tol
        assert np.max(np.abs(C_gpu - C_ref)) <= tol
    return res, C_ref


@pytest.mark.parametrize("n_rows,n_inner,n_cols,log2b,d", [
    (300, 77, 250, 13, 3),     # fused, b_lo = 2^13, one slice
    (129, 300, 64, 15, 5),     # fused, four slices, ragged
    (64, 33, 97, 11, 1),       # fused, smallest b_lo
    (50, 20, 40, 8, 3),        # composed path (b < 2^11)
    (1, 1, 1, 12, 3),          # degenerate 1x1x1
])
def test_estimate_integer_bit_exact(n_rows, n_inner, n_cols, log2b, d):
    announce(f"estimate int {n_rows}x{n_inner}x{n_cols} log2b={log2b} d={d}")
    w = small_random(n_rows, n_inner, n_cols, log2b, d, seed=n_rows + log2b, integer=True)
    _estimate_and_compare(w, n_rows, n_cols, exact=True)


@pytest.mark.parametrize("n_rows,n_inner,n_cols,log2b,d", [
    (300, 77, 250, 13, 3), (129, 300, 64, 15, 5), (50, 20, 40, 8, 3)])
def test_estimate_real_within_tolerance(n_rows, n_inner, n_cols, log2b, d):
    announce(f"estimate real {n_rows}x{n_inner}x{n_cols} log2b={log2b} d={d}")
    w = small_random(n_rows, n_inner, n_cols, log2b, d, seed=7 + log2b)
    _estimate_and_compare(w, n_rows, n_cols, exact=False)


def test_estimate_exact_sparse_256():
    announce("estimate hadamard n=256 b=2^12 d=5")
    w = exact_sparse_256(0)
    res, C_ref = _estimate_and_compare(w, 256, 256, exact=False)
    # recovered nonzeros: the GPU's set equals the oracle's
    tol = 1e-9 * np.linalg.norm(w.C_exact) / 256
    ok_gpu = np.abs(host(res.C_hat) - w.C_exact) <= tol
    ok_ref = np.abs(C_ref - w.C_exact) <= tol
    assert np.array_equal(ok_gpu, ok_ref)


def test_estimate_identity_tables_is_matmul():
    # h1(i) = i n, h2(j) = j, signs +1, b = n^2: the estimate is A B exactly.
    announce("estimate identity tables n=64")
    t = torch()
    n, log2b, d = 64, 12, 3
    rng = np.random.default_rng(4)
    A = rng.integers(-9, 10, (n, n)).astype(np.float64)
    B = rng.integers(-9, 10, (n, n)).astype(np.float64)
    t1 = np.tile((np.arange(n) * n).astype(np.uint32), (d, 1))
    t2 = np.tile(np.arange(n).astype(np.uint32), (d, 1))
    res = cmm.estimate(dev(A), dev(B), d, log2b, tab1=tables_dev(t1), tab2=tables_dev(t2))
    assert np.array_equal(host(res.C_hat), A @ B)


def test_estimate_deterministic():
    announce("estimate determinism")
    w = small_random(200, 150, 180, 14, 5, seed=99)
    A, B = dev(w.A), dev(w.B)
    r1 = cmm.estimate(A, B, w.d, w.log2b, keys=w.keys)
    r2 = cmm.estimate(A, B, w.d, w.log2b, keys=w.keys)
    assert torch().equal(r1.p, r2.p) and torch().equal(r1.C_hat, r2.C_hat)


def test_estimate_deterministic_full_size():
    # real-valued data at the headline shape (n = 4096, b = 2^16, d = 9):
    # collision sums, window reduce and k-range partials run in a fixed
    # order, so two runs agree bit for bit
    announce("estimate determinism n=4096 b=2^16 d=9 N(0,1)")
    rng = np.random.default_rng(4096)
    A = dev(rng.standard_normal((4096, 4096)))
    B = dev(rng.standard_normal((4096, 4096)))
    keys = draw_keys(9, 77)
    r1 = cmm.estimate(A, B, 9, 16, keys=keys)
    r2 = cmm.estimate(A, B, 9, 16, keys=keys)
    assert torch().equal(r1.p, r2.p) and torch().equal(r1.C_hat, r2.C_hat)


def test_estimate_f32_compute():
    announce("estimate f32 compute")
    w = small_random(256, 128, 200, 14, 5, seed=5)
    t = torch()
    res = cmm.estimate(dev(w.A.astype(np.float32)), dev(w.B.astype(np.float32)), w.d, w.log2b,
                       keys=w.keys, compute="f32")
    t1, t2 = O.hash_tables(w.keys, 256, 200, w.log2b)
    A32, B32 = w.A.astype(np.float32).astype(np.float64), w.B.astype(np.float32).astype(np.float64)
    C = O.product(A32, B32)
    p_ref = O.bucket_sums(C, t1, t2, w.log2b)
    C_ref = O.extract(p_ref, t1, t2, "median")
    # the float32 tolerance derived in tests/numerics.py (every butterfly
    # level and the accumulation over the 128 values of k round)
    tol = f32_tolerance(A32, B32, w.log2b, k_run=128)
    print(f"f32: max|dp| {np.abs(host(res.p) - p_ref).max() / tol:.3f} of tol", flush=True)
    assert np.max(np.abs(host(res.p) - p_ref)) <= tol
    assert np.max(np.abs(host(res.C_hat) - C_ref)) <= tol


def test_estimate_zero_inner_dimension():
    announce("estimate n_inner=0")
    t = torch()
    A = t.zeros((5, 0), dtype=t.float64, device="cuda")
    B = t.zeros((0, 7), dtype=t.float64, device="cuda")
    res = cmm.estimate(A, B, 3, 12, keys=draw_keys(3, 1))
    assert np.array_equal(host(res.C_hat), np.zeros((5, 7)))


def test_estimate_planted_4096_full_size_bit_exact():
    # The benchmark configuration, in the launch configuration bench.py uses.
    # All values are integers with every intermediate below 2^53 (|X|, |Y| <=
    # 4n = 2^14, sums over k <= 2^40, |p_hat| <= 2^40, inverse sums < 2^53),
    # so float64 results are exact and must match the oracle bit for bit.
    from workloads import planted_4096
    from workloads.metrics import planted_recall
    announce("estimate planted n=4096 b=2^16 d=9 (full size)")
    w = planted_4096(0)
    assert np.abs(w.A).max() * w.n * w.n * w.n < 2.0 ** 53
    res = cmm.estimate(dev(w.A), dev(w.B), w.d, w.log2b, keys=w.keys)
    t1, t2 = O.hash_tables(w.keys, w.n, w.n, w.log2b)
    p_ref = O.bucket_sums(O.product(w.A, w.B), t1, t2, w.log2b)
    assert np.array_equal(host(res.p), p_ref)
    C_gpu = host(res.C_hat)
    rows = np.arange(0, w.n, 7)           # sampled rows, all columns
    C_ref = O.extract(p_ref, t1, t2, "median", rows=rows)
    assert np.array_equal(C_gpu[rows], C_ref)
    rec = planted_recall(C_gpu, w.rows, w.cols, w.tau)
    assert rec["recall"] >= 4095 / 4096
