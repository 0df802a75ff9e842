"""Sparse queries on the GPU: Decompress at a list of entries against the
oracle, and heavy-hitter extraction against the dense extract (the same
values bit for bit, the same set of entries)."""
import numpy as np
import pytest

import oracle as O
import paper_2601_09477_amd as cmm
from workloads import planted_4096, small_random
from tests.gpu_util import announce, dev, host, tables_dev, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch().cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()


def _setup(nr, ni, nc, log2b, d, seed):
    w = small_random(nr, ni, nc, log2b, d, seed=seed)
    t1, t2 = O.hash_tables(w.keys, nr, nc, log2b)
    p = O.bucket_sums(O.product(w.A, w.B), t1, t2, log2b)
    return p, t1, t2


@pytest.mark.parametrize("d,est", [(5, "median"), (9, "median"), (13, "median"), (4, "mean"),
                                   (7, "mean")])
def test_extract_entries_matches_oracle(d, est):
    announce(f"extract entries d={d} {est}")
    T = torch()
    p, t1, t2 = _setup(120, 60, 90, 11, d, seed=d)
    rng = np.random.default_rng(d)
    rows = rng.integers(-3, 123, 1000)
    cols = rng.integers(-2, 92, 1000)
    want = O.extract_entries(p, t1, t2, rows, cols, est)
    code = cmm.CMM_MEDIAN if est == "median" else cmm.CMM_MEAN
    for dt in (T.float64, T.float32):
        out = T.empty(1000, dtype=dt, device="cuda")
        cmm.cmm_extract_entries(dev(p), tables_dev(t1), tables_dev(t2), d, 120, 90, 11, code,
                                dev(rows), dev(cols), out)
        got = host(out).astype(np.float64)
        assert np.array_equal(np.isnan(got), np.isnan(want))
        ok = ~np.isnan(want)
        if dt == T.float64:
            assert np.array_equal(got[ok], want[ok])
        else:
            assert np.array_equal(got[ok], want[ok].astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("d,est", [(5, "median"), (13, "median"), (4, "mean")])
def test_heavy_hitters_equal_dense_threshold(d, est):
    announce(f"heavy hitters d={d} {est}")
    T = torch()
    nr, nc, log2b = 300, 270, 12
    p, t1, t2 = _setup(nr, 80, nc, log2b, d, seed=20 + d)
    code = cmm.CMM_MEDIAN if est == "median" else cmm.CMM_MEAN
    pd, a, b = dev(p), tables_dev(t1), tables_dev(t2)
    C = T.empty((nr, nc), dtype=T.float64, device="cuda")
    cmm.cmm_extract(pd, a, b, d, nr, nc, log2b, code, C)
    Ch = host(C)
    for thr in (0.0, float(np.quantile(np.abs(Ch), 0.97)), float(np.abs(Ch).max()) * 2):
        cap = nr * nc
        rows = T.empty(cap, dtype=T.int64, device="cuda")
        cols = T.empty(cap, dtype=T.int64, device="cuda")
        vals = T.empty(cap, dtype=T.float64, device="cuda")
        count = T.full((1,), -5, dtype=T.int64, device="cuda")
        cmm.cmm_extract_heavy(pd, a, b, d, nr, nc, log2b, code, thr, rows, cols, vals, count)
        k = int(count.item())
        ri, ci = np.nonzero(np.abs(Ch) >= thr)
        assert k == len(ri)
        r, c, v = host(rows)[:k], host(cols)[:k], host(vals)[:k]
        order = np.lexsort((c, r))
        assert np.array_equal(r[order], ri) and np.array_equal(c[order], ci)
        assert np.array_equal(v[order], Ch[ri, ci])


def test_heavy_hitters_capacity_overflow():
    announce("heavy hitters capacity")
    T = torch()
    nr, nc, log2b, d = 200, 150, 11, 5
    p, t1, t2 = _setup(nr, 50, nc, log2b, d, seed=3)
    pd, a, b = dev(p), tables_dev(t1), tables_dev(t2)
    C = T.empty((nr, nc), dtype=T.float64, device="cuda")
    cmm.cmm_extract(pd, a, b, d, nr, nc, log2b, cmm.CMM_MEDIAN, C)
    Ch = host(C)
    cap = 100
    rows = T.full((cap,), -1, dtype=T.int64, device="cuda")
    cols = T.full((cap,), -1, dtype=T.int64, device="cuda")
    vals = T.empty(cap, dtype=T.float32, device="cuda")
    count = T.zeros(1, dtype=T.int64, device="cuda")
    cmm.cmm_extract_heavy(pd, a, b, d, nr, nc, log2b, cmm.CMM_MEDIAN, 0.0, rows, cols, vals, count)
    assert int(count.item()) == nr * nc
    r, c, v = host(rows), host(cols), host(vals)
    assert np.all((r >= 0) & (r < nr) & (c >= 0) & (c < nc))
    assert len(set(zip(r.tolist(), c.tolist()))) == cap
    assert np.array_equal(v, Ch[r, c].astype(np.float32))


def test_heavy_hitters_planted_4096_full_size():
    """n = 4096, b = 2^16, d = 9: the heavy hitters above tau = 2n straight
    from the sketch equal the thresholded dense estimate, and hold every
    planted pair."""
    from workloads.metrics import planted_recall
    announce("heavy hitters planted n=4096")
    T = torch()
    w = planted_4096(0)
    res = cmm.estimate(dev(w.A), dev(w.B), w.d, w.log2b, keys=w.keys)
    r, c, v = cmm.heavy_hitters(res, w.tau)
    Ch = host(res.C_hat)
    ri, ci = np.nonzero(np.abs(Ch) >= w.tau)
    assert np.array_equal(host(r), ri) and np.array_equal(host(c), ci)
    assert np.array_equal(host(v), Ch[ri, ci])
    rec = planted_recall(Ch, w.rows, w.cols, w.tau)
    hits = set(zip(host(r).tolist(), host(c).tolist()))
    assert sum((int(i), int(j)) in hits for i, j in zip(w.rows, w.cols)) == rec["recalled"]
    assert rec["recalled"] == rec["planted"]
