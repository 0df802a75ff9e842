"""The standalone steps at the bench's unfused configuration: n = 4096,
b = 2^16, d = 9, a chunk of 64 values of k, the planted +-1 inputs.  Each
step's output is compared with the oracle on sampled slices (GPU).  The
data are integers well below 2^53, so every comparison is exact."""
import numpy as np
import pytest

import oracle as O
import paper_2601_09477_amd as cmm
from workloads import planted_4096
from tests.gpu_util import announce, dev, host, tables_dev, torch

pytestmark = pytest.mark.gpu

KC = 64
SAMPLE_K = (0, 37, 63)


@pytest.fixture(scope="module")
def chunk():
    T = torch()
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()
    w = planted_4096(0)
    t1, t2 = O.hash_tables(w.keys, w.n, w.n, w.log2b)
    d, b = w.d, 1 << w.log2b
    X = T.empty((d, KC, b), dtype=T.float64, device="cuda")
    Y = T.empty((d, KC, b), dtype=T.float64, device="cuda")
    cmm.cmm_sketch(0, dev(w.A), w.n, w.n, w.n, tables_dev(t1), d, w.log2b, 0, KC, X)
    cmm.cmm_sketch(1, dev(w.B), w.n, w.n, w.n, tables_dev(t2), d, w.log2b, 0, KC, Y)
    T.cuda.synchronize()
    return w, t1, t2, X, Y


def test_sketch_full_size_sampled(chunk):
    w, t1, t2, X, Y = chunk
    announce("sketch full size n=4096 b=2^16 d=9 kc=64 (sampled k)")
    for side, M, tab, S in ((0, w.A, t1, X), (1, w.B, t2, Y)):
        got = host(S)
        for kk in SAMPLE_K:
            want = O.count_sketch(M, tab, side, kk, 1, w.log2b)[:, 0, :]
            assert np.array_equal(got[:, kk, :], want), (side, kk)


def test_fwht_accumulate_full_size_sampled(chunk):
    w, t1, t2, X, Y = chunk
    T = torch()
    announce("fwht + accumulate full size, 576 vectors of 2^16 (sampled)")
    d, b = w.d, 1 << w.log2b
    Xs, Ys = host(X), host(Y)
    Xt, Yt = X.clone(), Y.clone()
    cmm.cmm_fwht(Xt, d * KC, w.log2b, 1.0)
    cmm.cmm_fwht(Yt, d * KC, w.log2b, 1.0)
    T.cuda.synchronize()
    Xh, Yh = host(Xt), host(Yt)
    for t, kk in ((0, 0), (4, 37), (8, 63)):
        assert np.array_equal(Xh[t, kk], O.wht(Xs[t, kk][None, :])[0]), (t, kk)
        assert np.array_equal(Yh[t, kk], O.wht(Ys[t, kk][None, :])[0]), (t, kk)
    p_hat = T.zeros((d, b), dtype=T.float64, device="cuda")
    cmm.cmm_accumulate(Xt, Yt, d, KC, w.log2b, p_hat)
    # inverse of one repetition's sum: 2^-m H H x = x
    back = p_hat[2:3].clone()
    cmm.cmm_fwht(back, 1, w.log2b, 1.0)
    cmm.cmm_fwht(back, 1, w.log2b, 2.0 ** -w.log2b)
    T.cuda.synchronize()
    us = np.random.default_rng(5).choice(b, size=257, replace=False)
    want = O.accumulate(Xh[:, :, us], Yh[:, :, us])
    ph = host(p_hat)
    assert np.array_equal(ph[:, us], want)
    assert np.array_equal(host(back)[0], ph[2])
