"""The evaluation protocol on the GPU: per-repetition estimates
(cmm_extract_reps) and the mean estimator over many repetitions against the
oracle, the correctness counters of Section 5.4 (cmm_correctness_counts)
against the oracle's counts, and the variance experiment of Section 5.3 as
a statistical check on every instance family."""
import math

import numpy as np
import pytest

import oracle as O
import paper_2601_09477_amd as cmm
from workloads import draw_keys, small_random
from workloads import instances as I
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
    return O.bucket_sums(O.product(w.A, w.B), t1, t2, log2b), t1, t2


@pytest.mark.parametrize("d", [1, 5, 1000])
def test_extract_reps_matches_oracle(d):
    announce(f"extract reps d={d}")
    T = torch()
    p, t1, t2 = _setup(90, 40, 70, 10, d, seed=d)
    rng = np.random.default_rng(d)
    rows = rng.integers(-2, 92, 300)
    cols = rng.integers(-1, 71, 300)
    want = O.extract_reps(p, t1, t2, rows, cols)
    for dt in (T.float64, T.float32):
        out = T.empty((d, 300), dtype=dt, device="cuda")
        cmm.cmm_extract_reps(dev(p), tables_dev(t1), tables_dev(t2), d, 90, 70, 10, dev(rows),
                             dev(cols), out)
        got = host(out).astype(np.float64)
        assert np.array_equal(np.isnan(got), np.isnan(want))
        ok = ~np.isnan(want)
        ref = want if dt == T.float64 else want.astype(np.float32).astype(np.float64)
        assert np.array_equal(got[ok], ref[ok])


def test_mean_over_many_repetitions():
    # d above the median's limit: dense extract, entries and heavy hitters
    # with the mean estimator against the oracle
    announce("mean estimator d=100")
    T = torch()
    d, nr, nc, log2b = 100, 70, 60, 9
    p, t1, t2 = _setup(nr, 30, nc, log2b, d, seed=8)
    want = O.extract(p, t1, t2, "mean")
    pd, a, b = dev(p), tables_dev(t1), tables_dev(t2)
    C = T.empty((nr, nc), dtype=T.float64, device="cuda")
    cmm.cmm_extract(pd, a, b, d, nr, nc, log2b, cmm.CMM_MEAN, C)
    assert np.abs(host(C) - want).max() <= 1e-12 * np.abs(want).max()
    rows = T.arange(nr, device="cuda", dtype=T.int64)
    cols = (rows * 7) % nc
    e = T.empty(nr, dtype=T.float64, device="cuda")
    cmm.cmm_extract_entries(pd, a, b, d, nr, nc, log2b, cmm.CMM_MEAN, rows, cols, e)
    assert np.array_equal(host(e), host(C)[host(rows), host(cols)])
    cap = nr * nc
    hr = T.empty(cap, dtype=T.int64, device="cuda")
    hc = T.empty(cap, dtype=T.int64, device="cuda")
    hv = T.empty(cap, dtype=T.float64, device="cuda")
    cnt = T.zeros(1, dtype=T.int64, device="cuda")
    thr = float(np.quantile(np.abs(host(C)), 0.9))
    cmm.cmm_extract_heavy(pd, a, b, d, nr, nc, log2b, cmm.CMM_MEAN, thr, hr, hc, hv, cnt)
    k = int(cnt.item())
    Ch = host(C)
    assert k == np.count_nonzero(np.abs(Ch) >= thr)
    assert np.array_equal(host(hv)[:k], Ch[host(hr)[:k], host(hc)[:k]])


@pytest.mark.parametrize("family", I.FAMILIES)
def test_correctness_counts_match_oracle(family):
    announce(f"correctness counts {family}")
    T = torch()
    n, log2b, d = 256, 11, 5
    w = I.instance(family, n, 11)
    A, B = host(w.A), host(w.B)
    C = O.product(A, B)
    keys = draw_keys(d, 606)
    br, bc = host(w.big_rows), host(w.big_cols)
    for out_dtype in (T.float64, T.float32):
        res = cmm.estimate(dev(A), dev(B), d, log2b, keys=keys, out_dtype=out_dtype)
        Ch = host(res.C_hat).astype(np.float64)
        for thr, tol in ((0.5, 0.1), (0.05, 0.01)):
            counts = T.full((4,), -1, dtype=T.int64, device="cuda")
            cmm.cmm_correctness_counts(res.C_hat, dev(C), dev(br), dev(bc), counts, thr, tol)
            assert host(counts).tolist() == O.correctness_counts(Ch, C, br, bc, thr, tol).tolist()


def test_correctness_counts_strided_and_out_of_range():
    announce("correctness counts strided")
    T = torch()
    rng = np.random.default_rng(1)
    C = rng.standard_normal((300, 280)) * 0.3
    Ch = C + rng.standard_normal(C.shape) * 0.08
    big_Ch = T.zeros((300, 300), dtype=T.float64, device="cuda")
    big_Ch[:, :280] = dev(Ch)
    big_C = T.zeros((300, 290), dtype=T.float64, device="cuda")
    big_C[:, :280] = dev(C)
    br = np.array([0, 299, 17, 400, -1])
    bc = np.array([0, 279, 5, 3, 2])
    counts = T.empty(4, dtype=T.int64, device="cuda")
    cmm.cmm_correctness_counts(big_Ch[:, :280], big_C[:, :280], dev(br), dev(bc), counts)
    want = O.correctness_counts(Ch, C, br[:3], bc[:3])
    assert host(counts).tolist() == want.tolist()


@pytest.mark.parametrize("family", I.FAMILIES)
def test_variance_experiment(family):
    """Section 5.3 at n = 256: 1000 independent draws (one per repetition,
    d = 1 each) of the estimate of a big entry, for two values of b: the
    mean is unbiased and the sample variance within the bound
    ||C||_F^2 / b of Pagh's Theorem 3.1; the first 20 draws equal the
    oracle's values."""
    announce(f"variance experiment {family}")
    T = torch()
    n, draws = 256, 1000
    w = I.instance(family, n, 21)
    A, B = host(w.A), host(w.B)
    C = O.product(A, B)
    i, j = int(host(w.big_rows)[0]), int(host(w.big_cols)[0])
    for log2b in (9, 12):
        keys = draw_keys(draws, 9000 + log2b)
        res = cmm.estimate(dev(A), dev(B), draws, log2b, keys=keys, estimator="mean",
                           dense=False)
        x = T.empty((draws, 1), dtype=T.float64, device="cuda")
        ri = T.tensor([i], dtype=T.int64, device="cuda")
        ci = T.tensor([j], dtype=T.int64, device="cuda")
        cmm.cmm_extract_reps(res.p, res.tab1, res.tab2, draws, n, n, log2b, ri, ci, x)
        xs = host(x)[:, 0]
        b = 1 << log2b
        bound = (np.linalg.norm(C) ** 2 - C[i, j] ** 2) / b
        assert abs(xs.mean() - C[i, j]) <= 4.5 * math.sqrt(bound / draws) + 1e-12, (log2b, xs.mean())
        # sampling noise of the variance: x - c is a signed sum of the
        # entries that collide with (i, j), each with probability 1 / b, so
        # (x - c)^2 has variance about sum c^4 / b (rare collisions) plus
        # 2 bound^2 (many collisions, the Gaussian regime)
        c4 = (np.sum(C ** 4) - C[i, j] ** 4) / b
        noise = math.sqrt((c4 + 2 * bound ** 2) / draws)
        assert xs.var() <= bound + 4 * noise + 1e-20, (log2b, xs.var(), bound, noise)
        t1, t2 = O.hash_tables(keys[:20], n, n, log2b)
        p20 = O.bucket_sums(C, t1, t2, log2b)
        ref = O.extract_reps(p20, t1, t2, [i], [j])[:, 0]
        scale = np.linalg.norm(C) / n
        assert np.abs(xs[:20] - ref).max() <= 1e-9 * scale
