"""One estimate captured in a HIP graph (GPU).

Every launch of cmm_estimate (hash, plans, the precision form's merged-chain
pre-pass, compress, partial sums, inverse transform, extract) goes into the
graph; no step may record a memset or depend on host state that changes
between replays.  Each replay, with poisoned outputs before it and eager
estimates on another workspace in between, must reproduce the eager result
bit for bit."""
import numpy as np
import pytest

import paper_2601_09477_amd as cmm
from workloads import draw_keys
from tests.gpu_util import announce, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch().cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()


def _setup(T, A, B, d, log2b, keys, compute):
    dev = A.device
    n_rows, n_cols = A.shape[0], B.shape[1]
    tab1 = T.empty((d, n_rows), dtype=T.int32, device=dev)
    tab2 = T.empty((d, n_cols), dtype=T.int32, device=dev)
    p = T.empty((d, 1 << log2b), dtype=T.float64, device=dev)
    C_hat = T.empty((n_rows, n_cols), dtype=T.float64, device=dev)
    pr = cmm.make_problem(A, B, d, log2b, keys=cmm.keys_tensor(keys, dev), tab1=tab1, tab2=tab2,
                          p=p, C_hat=C_hat, compute=compute)
    nbytes = cmm.cmm_workspace_size(pr)
    ws = T.empty(max(nbytes, 1), dtype=T.uint8, device=dev)
    return pr, ws, nbytes, p, C_hat


@pytest.mark.parametrize("compute,log2b", [("f64", 13), ("f32", 13), ("bf16", 14)])
def test_estimate_graph_replays(compute, log2b):
    announce(f"estimate graph capture {compute} log2b={log2b}")
    T = torch()
    rng = np.random.default_rng(7)
    n_rows, n_inner, n_cols, d = 1000, 192, 904, 5
    A = T.from_numpy(rng.integers(-1, 2, size=(n_rows, n_inner)).astype(np.float64)).cuda()
    B = T.from_numpy(rng.integers(-1, 2, size=(n_inner, n_cols)).astype(np.float64)).cuda()
    keys = draw_keys(d, 99)
    pr, ws, nbytes, p, C_hat = _setup(T, A, B, d, log2b, keys, compute)
    pr2, ws2, nbytes2, p2, C2 = _setup(T, A, B, d, log2b, keys, compute)
    stream = T.cuda.current_stream()
    cmm.cmm_estimate(pr, ws, nbytes, stream)
    T.cuda.synchronize()
    want_p, want_C = p.clone(), C_hat.clone()
    s = T.cuda.Stream()
    s.wait_stream(stream)
    with T.cuda.stream(s):
        cmm.cmm_estimate(pr, ws, nbytes, s)   # warm up on the capture stream
    stream.wait_stream(s)
    T.cuda.synchronize()
    g = T.cuda.CUDAGraph()
    with T.cuda.graph(g):
        cmm.cmm_estimate(pr, ws, nbytes, T.cuda.current_stream())
    T.cuda.synchronize()
    for rep in range(3):
        p.fill_(float("nan"))
        C_hat.fill_(12345.0)
        ws.fill_(0xA5)
        g.replay()
        T.cuda.synchronize()
        assert T.equal(p, want_p), rep
        assert T.equal(C_hat, want_C), rep
        cmm.cmm_estimate(pr2, ws2, nbytes2, stream)   # eager work between replays
        T.cuda.synchronize()
        assert T.equal(p2, want_p), rep
