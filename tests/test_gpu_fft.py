"""Pagh's FFT form on the GPU: the batched transform against numpy.fft, the
cyclic Decompress against the oracle (bit-exact from the same p), and the
end-to-end FFT-form estimate against the oracle's plain definition."""
import numpy as np
import pytest

import oracle as O
import paper_2601_09477_amd as cmm
from workloads import draw_keys, planted_4096, small_random
from tests.gpu_util import announce, dev, host, tables_dev, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch().cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()


@pytest.mark.parametrize("log2n,batch", [(1, 3), (5, 7), (12, 2), (13, 3), (16, 2), (20, 1)])
@pytest.mark.parametrize("inverse", [False, True])
def test_fft_matches_numpy(log2n, batch, inverse):
    announce(f"fft log2n={log2n} batch={batch} inverse={inverse}")
    T = torch()
    rng = np.random.default_rng(log2n)
    n = 1 << log2n
    x = rng.standard_normal((batch, n)) + 1j * rng.standard_normal((batch, n))
    scale = 2.0 ** -log2n if inverse else 1.0
    want = np.fft.ifft(x, axis=-1) if inverse else np.fft.fft(x, axis=-1)
    xd = dev(x)
    out = T.empty_like(xd)
    cmm.cmm_fft(xd, out, inverse=inverse, scale=scale)
    got = host(out)
    # float64 FFT rounding: about eps log2 n of the vector norm per entry
    norm = np.linalg.norm(x, axis=-1).max() * (scale if inverse else 1.0)
    assert np.abs(got - want).max() <= 4e-16 * (log2n + 1) * norm
    if log2n <= 12:    # in place
        cmm.cmm_fft(xd, xd, inverse=inverse, scale=scale)
        assert T.equal(xd, out)


def test_extract_cyclic_bit_exact():
    announce("extract cyclic")
    T = torch()
    w = small_random(130, 40, 150, 11, 5, seed=6)
    t1, t2 = O.hash_tables(w.keys, 130, 150, 11)
    p = O.bucket_sums_cyclic(O.product(w.A, w.B), t1, t2, 11)
    for est in ("median", "mean"):
        want = O.extract_cyclic(p, t1, t2, est)
        C = T.empty((130, 150), dtype=T.float64, device="cuda")
        code = cmm.CMM_MEDIAN if est == "median" else cmm.CMM_MEAN
        cmm.cmm_extract_cyclic(dev(p), tables_dev(t1), tables_dev(t2), 5, 130, 150, 11, code, C)
        if est == "median":
            assert np.array_equal(host(C), want)
        else:
            assert np.abs(host(C) - want).max() <= 1e-15 * np.abs(want).max()


# (n_rows, n_inner, n_cols, log2b, d): ragged shapes, b from 2^9 to 2^16
# (single-pass and two-pass transforms), several k-chunks at 2^16
SHAPES = [(37, 23, 41, 9, 3), (120, 64, 90, 12, 1), (200, 70, 130, 13, 5),
          (64, 150, 80, 16, 5)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("integer", [True, False])
def test_estimate_fft_matches_oracle(shape, integer):
    nr, ni, nc, log2b, d = shape
    announce(f"estimate fft {shape} integer={integer}")
    w = small_random(nr, ni, nc, log2b, d, seed=sum(shape), integer=integer)
    t1, t2 = O.hash_tables(w.keys, nr, nc, log2b)
    C = O.product(w.A, w.B)
    p_ref = O.bucket_sums_cyclic(C, t1, t2, log2b)
    res = cmm.estimate_fft(dev(w.A), dev(w.B), d, log2b, keys=w.keys)
    assert np.array_equal(cmm.tables_to_numpy(res.tab1), t1)
    p = host(res.p)
    # the transform route rounds: float64, O(eps log2 b) of the sketch norms
    scale = np.linalg.norm(C) / ni
    assert np.abs(p - p_ref).max() <= 1e-9 * scale
    if integer:
        assert np.array_equal(np.rint(p), p_ref)
    C_ref = O.extract_cyclic(p_ref, t1, t2, "median")
    assert np.abs(host(res.C_hat) - C_ref).max() <= 1e-9 * scale


def test_estimate_fft_degenerate_and_tables():
    announce("estimate fft degenerate")
    T = torch()
    w = small_random(30, 0, 20, 10, 3, seed=1)
    A = T.zeros((30, 0), dtype=T.float64, device="cuda")
    B = T.zeros((0, 20), dtype=T.float64, device="cuda")
    res = cmm.estimate_fft(A, B, 3, 10, keys=w.keys)
    assert np.all(host(res.p) == 0) and np.all(host(res.C_hat) == 0)
    # explicit tables (another family) instead of keys
    w = small_random(50, 30, 40, 12, 3, seed=2, integer=True)
    from workloads import draw_family_keys
    keys = draw_family_keys("tabulation", 3, 77)
    tab1, tab2 = cmm.family_tables("tabulation", keys, 50, 40, 12)
    res = cmm.estimate_fft(dev(w.A), dev(w.B), 3, 12, tab1=tab1, tab2=tab2, estimator="mean")
    t1, t2 = O.hash_tables_family("tabulation", keys, 50, 40, 12)
    p_ref = O.bucket_sums_cyclic(O.product(w.A, w.B), t1, t2, 12)
    assert np.array_equal(np.rint(host(res.p)), p_ref)


def test_estimate_fft_planted_4096_full_size():
    """n = 4096, b = 2^16, d = 9: the FFT form on the headline workload.
    Every entry of p against the oracle's cyclic bucket sums of the exact
    integer product: the float64 transform's rounding stays far below 1/2,
    so p rounds to the oracle's integers exactly; C_hat on every 37th row
    against the oracle's cyclic Decompress; every planted pair recalled."""
    from workloads.metrics import planted_recall
    announce("estimate fft planted n=4096")
    w = planted_4096(0)
    res = cmm.estimate_fft(dev(w.A), dev(w.B), w.d, w.log2b, keys=w.keys)
    p = host(res.p)
    t1, t2 = O.hash_tables(w.keys, 4096, 4096, w.log2b)
    p_ref = O.bucket_sums_cyclic(O.product(w.A, w.B), t1, t2, w.log2b)
    dp = np.abs(p - p_ref).max()
    print(f"fft full size: max|p - p_ref| = {dp:.3e}", flush=True)
    assert dp < 1e-6
    assert np.array_equal(np.rint(p), p_ref)
    rows = np.arange(0, 4096, 37)
    C_ref = O.extract_cyclic(p_ref, t1[:, rows], t2, "median")
    assert np.abs(host(res.C_hat)[rows] - C_ref).max() < 1e-6
    rec = planted_recall(host(res.C_hat), w.rows, w.cols, w.tau)
    assert rec["recalled"] == rec["planted"]
