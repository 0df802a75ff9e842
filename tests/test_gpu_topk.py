"""Top-K Decompress (cmm_extract_topk) against the oracle (GPU): the k
entries of largest |C_hat| without the dense output, sorted by magnitude
with ties broken by the smaller row-major index.  Rows, columns and values
must equal those of the oracle's dense Decompress followed by a plain sort,
bit for bit (the estimates are exact selections of p values, or sums in
repetition order for the mean)."""
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


def _check(res, t1, t2, n_rows, n_cols, k, estimator, dtype=None):
    T = torch()
    rows, cols, vals = cmm.topk(res, n_rows, n_cols, k, estimator, dtype=dtype)
    T.cuda.synchronize()
    r_ref, c_ref, v_ref = O.extract_topk(host(res.p), t1, t2, k, estimator)
    assert np.array_equal(host(rows), r_ref)
    assert np.array_equal(host(cols), c_ref)
    if dtype == T.float32:
        assert np.array_equal(host(vals), v_ref.astype(np.float32))
    else:
        assert np.array_equal(host(vals), v_ref)


@pytest.mark.parametrize("shape", [(300, 40, 257, 11, 5), (64, 30, 1000, 12, 3),
                                   (513, 20, 31, 10, 7), (40, 8, 40, 13, 1)])
def test_topk_small_integer_ties(shape):
    # small integer operands: many estimates tie, so the index order matters
    nr, ni, nc, log2b, d = shape
    announce(f"topk small integer {shape}")
    w = small_random(nr, ni, nc, log2b, d, seed=nr + nc, integer=True)
    res = cmm.estimate(dev(w.A), dev(w.B), d, log2b, keys=w.keys)
    t1, t2 = O.hash_tables(w.keys, nr, nc, log2b)
    for k in (1, 13, 1000, nr * nc):
        k = min(k, nr * nc)
        _check(res, t1, t2, nr, nc, k, "median")
    _check(res, t1, t2, nr, nc, 777, "mean")
    _check(res, t1, t2, nr, nc, 500, "median", dtype=torch().float32)


def test_topk_all_ties_resolves_every_level():
    # every estimate is zero: the magnitudes all tie and the selection runs
    # through all eight digit levels down to the index
    announce("topk all ties")
    T = torch()
    n_rows, n_cols, d, log2b = 70, 90, 3, 10
    p = T.zeros((d, 1 << log2b), dtype=T.float64, device="cuda")
    t1, t2 = O.hash_tables(draw_keys(d, 5), n_rows, n_cols, log2b)
    res = cmm.Estimate(None, p, tables_dev(t1), tables_dev(t2))
    for k in (1, 100, 4321, n_rows * n_cols):
        rows, cols, vals = cmm.topk(res, n_rows, n_cols, k)
        T.cuda.synchronize()
        idx = host(rows) * n_cols + host(cols)
        assert np.array_equal(idx, np.arange(k))
        assert np.all(host(vals) == 0.0)


def test_topk_argument_checks():
    announce("topk argument checks")
    T = torch()
    w = small_random(20, 5, 30, 9, 3, seed=3)
    res = cmm.estimate(dev(w.A), dev(w.B), 3, 9, keys=w.keys)
    with pytest.raises(cmm.CmmError):
        cmm.topk(res, 20, 30, 20 * 30 + 1)          # more than the block holds
    rows = T.empty(0, dtype=T.int64, device="cuda")
    vals = T.empty(0, dtype=T.float64, device="cuda")
    cmm.cmm_extract_topk(res.p, res.tab1, res.tab2, 3, 20, 30, 9, cmm.CMM_MEDIAN, 0, rows, rows,
                         vals)                          # k = 0: nothing to do


@pytest.mark.parametrize("k", [4096, 20000])
def test_topk_planted_4096_full_size(k):
    # the benchmark workload (n = 4096, b = 2^16, d = 9): the top-k against
    # the oracle's dense Decompress and sort, and for k = 4096 the planted
    # pairs' share of it
    from workloads.metrics import planted_recall
    announce(f"topk planted n=4096 k={k}")
    w = planted_4096(0)
    res = cmm.estimate(dev(w.A), dev(w.B), w.d, w.log2b, keys=w.keys, dense=False)
    t1, t2 = O.hash_tables(w.keys, w.n, w.n, w.log2b)
    rows, cols, vals = cmm.topk(res, w.n, w.n, k)
    torch().cuda.synchronize()
    r_ref, c_ref, v_ref = O.extract_topk(host(res.p), t1, t2, k, "median")
    assert np.array_equal(host(rows), r_ref)
    assert np.array_equal(host(cols), c_ref)
    assert np.array_equal(host(vals), v_ref)
    if k == 4096:
        got = set(zip(host(rows).tolist(), host(cols).tolist()))
        planted = set(zip(w.rows.tolist(), w.cols.tolist()))
        print(f"top-4096 holds {len(got & planted)} of the 4096 planted pairs", flush=True)
