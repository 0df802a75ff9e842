"""Batched form on the GPU: many problems of uneven size in one persistent
Compress launch, checked problem by problem against the oracle; every
launch configuration of the tuner; degenerate problems inside a batch; graph
capture and replay; the autotuner and its cache; the full 64-pair mix."""
import numpy as np
import pytest

import oracle as O
import paper_2601_09477_amd as cmm
from workloads import batched_mix, draw_keys
from workloads.metrics import planted_recall
from tests.gpu_util import announce, dev, host, torch
from tests.numerics import f32_tolerance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch().cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()


# (n_rows, n_inner, n_cols, log2b, d): ragged, b_hi from 1 to 8 at b_lo = 2^13
# (every b_lo from 2^11 to 2^13 is a candidate for these)
SHAPES = [(64, 48, 80, 13, 3), (300, 130, 200, 14, 5), (128, 256, 96, 16, 3),
          (17, 9, 33, 13, 3), (256, 200, 256, 15, 7), (90, 64, 40, 13, 5)]


def _problems(shapes, integer, seed, dtype=np.float64):
    rng = np.random.default_rng(seed)
    out = []
    for q, (nr, ni, nc, lb, d) in enumerate(shapes):
        if integer:
            A = rng.integers(-3, 4, size=(nr, ni)).astype(np.float64)
            B = rng.integers(-3, 4, size=(ni, nc)).astype(np.float64)
        else:
            A = rng.standard_normal((nr, ni))
            B = rng.standard_normal((ni, nc))
        out.append((A, B, d, lb, draw_keys(d, 5000 + 10 * seed + q)))
    return out


def _oracle(A, B, d, log2b, keys):
    t1, t2 = O.hash_tables(keys, A.shape[0], B.shape[1], log2b)
    C = O.product(A, B)
    p = O.bucket_sums(C, t1, t2, log2b)
    return C, p, O.extract(p, t1, t2, "median"), t1, t2


def _device_batch(probs, compute, dtype):
    t = torch()
    pairs = [(dev(A, dtype), dev(B, dtype), d, lb, keys) for A, B, d, lb, keys in probs]
    batch, res = cmm.make_batch(pairs, compute=compute)
    return batch, res, pairs


def test_batched_f64_integer_bit_exact_every_config():
    announce("batched f64 integer, every configuration")
    probs = _problems(SHAPES, True, 1)
    refs = [_oracle(*p) for p in probs]
    batch, res, _ = _device_batch(probs, "f64", torch().float64)
    ws = batch.workspace()
    configs = [(lb, kg, wg, o, r) for lb in (11, 12, 13) for kg in (32, 64, 128, 256)
               for wg in (1, 2) for o in (0, 1) for r in (16, 32) if r == 32 or lb == 13]
    for cfg in configs:
        announce(f"batched f64 config {cfg}")
        batch.set_config(*cfg)
        batch.run(ws)
        torch().cuda.synchronize()
        for q, (C, p, C_hat, t1, t2) in enumerate(refs):
            assert np.array_equal(cmm.tables_to_numpy(res[q].tab1), t1)
            assert np.array_equal(host(res[q].p), p), (cfg, q)
            assert np.array_equal(host(res[q].C_hat), C_hat), (cfg, q)


def test_batched_f32_matches_oracle():
    announce("batched f32 real")
    probs = _problems(SHAPES, False, 2)
    batch, res, _ = _device_batch(probs, "f32", torch().float32)
    ws = batch.workspace()
    batch.run(ws)
    torch().cuda.synchronize()
    for q, (A, B, d, lb, keys) in enumerate(probs):
        A32 = A.astype(np.float32).astype(np.float64)
        B32 = B.astype(np.float32).astype(np.float64)
        C, p, C_hat, t1, t2 = _oracle(A32, B32, d, lb, keys)
        tol = f32_tolerance(A32, B32, lb, k_run=max(1, A.shape[1]))
        assert np.max(np.abs(host(res[q].p) - p)) <= tol, q
        assert np.max(np.abs(host(res[q].C_hat) - C_hat)) <= tol, q


def test_batched_degenerate_problems():
    # an empty inner dimension (C_hat = 0) and an empty row range inside a batch
    announce("batched degenerate")
    probs = _problems([(40, 32, 50, 12, 3), (30, 0, 20, 12, 3), (0, 16, 24, 11, 3),
                       (70, 20, 10, 13, 5)], True, 3)
    refs = [_oracle(*p) for p in probs]
    batch, res, _ = _device_batch(probs, "f64", torch().float64)
    ws = batch.workspace()
    batch.run(ws)
    torch().cuda.synchronize()
    for q, (C, p, C_hat, t1, t2) in enumerate(refs):
        assert np.array_equal(host(res[q].p), p), q
        if res[q].C_hat.numel():
            assert np.array_equal(host(res[q].C_hat), C_hat), q


def test_batched_graph_capture_replays():
    # Captured once; every replay (with eager runs of the same batch on
    # another workspace, and garbage written to the outputs, in between)
    # reproduces the eager result bit for bit.
    announce("batched graph capture")
    T = torch()
    probs = _problems(SHAPES[:4], False, 4)
    batch, res, _ = _device_batch(probs, "f32", T.float32)
    ws, ws2 = batch.workspace(), batch.workspace()
    batch.run(ws)
    T.cuda.synchronize()
    want = [(r.p.clone(), r.C_hat.clone()) for r in res]
    s = T.cuda.Stream()
    s.wait_stream(T.cuda.current_stream())
    with T.cuda.stream(s):
        batch.run(ws)   # warm up on the capture stream
    T.cuda.current_stream().wait_stream(s)
    T.cuda.synchronize()
    g = T.cuda.CUDAGraph()
    with T.cuda.graph(g):
        batch.run(ws)
    T.cuda.synchronize()
    for rep in range(3):
        for r in res:
            r.p.fill_(float("nan"))
            r.C_hat.fill_(12345.0)
        g.replay()
        T.cuda.synchronize()
        for q, r in enumerate(res):
            assert T.equal(r.p, want[q][0]), (rep, q)
            assert T.equal(r.C_hat, want[q][1]), (rep, q)
        batch.run(ws2)   # eager work between replays
        T.cuda.synchronize()
        for q, r in enumerate(res):
            assert T.equal(r.p, want[q][0]), (rep, q)


def test_batched_autotune_and_cache():
    announce("batched autotune")
    probs = _problems(SHAPES[:3], True, 5)
    refs = [_oracle(*p) for p in probs]
    batch, res, _ = _device_batch(probs, "f64", torch().float64)
    ws = batch.workspace()
    cfg = batch.autotune(ws)
    assert cfg["source"] in ("tuned", "cache")
    batch.run(ws)
    torch().cuda.synchronize()
    for q, (C, p, C_hat, t1, t2) in enumerate(refs):
        assert np.array_equal(host(res[q].p), p)
    # a second batch with the same signature takes the cached choice
    batch2, res2, _ = _device_batch(probs, "f64", torch().float64)
    cfg2 = batch2.autotune(batch2.workspace())
    assert cfg2["source"] == "cache"
    keys = ("log2_blo", "k_per_item", "wg_per_cu", "order", "radix")
    assert {k: cfg2[k] for k in keys} == {k: cfg[k] for k in keys}


def test_batched_mix_64_pairs_full_size():
    """64 pairs, n uniform over {512, 1024, 2048, 4096}, b = 16 n, d = 7,
    float32: every exactly-sparse pair against the oracle's bucket sums of
    its exact product; every planted pair's heavy hitters recovered (or
    missed exactly where the oracle's estimate misses them); the smallest
    and the largest planted pair against the full oracle."""
    announce("batched mix 64 pairs")
    T = torch()
    ws_list = batched_mix(0)
    pairs = [(dev(w.A, T.float32), dev(w.B, T.float32), w.d, w.log2b, w.keys) for w in ws_list]
    batch, res = cmm.make_batch(pairs, compute="f32")
    ws = batch.workspace()
    batch.run(ws)
    T.cuda.synchronize()
    planted = []
    for q, w in enumerate(ws_list):
        t1 = cmm.tables_to_numpy(res[q].tab1)
        t2 = cmm.tables_to_numpy(res[q].tab2)
        if w.kind == "exact":
            r, c = np.nonzero(w.C_exact)
            p_ref = O.bucket_sums_sparse(r, c, w.C_exact[r, c], t1, t2, w.log2b)
            # float32 copies of the real operand B count as one more rounding level
            tol = f32_tolerance(w.A, w.B, w.log2b, k_run=w.n, operands_rounded=False)
            assert np.max(np.abs(host(res[q].p) - p_ref)) <= tol, q
            rows = np.arange(0, w.n, max(1, w.n // 64))
            C_ref = O.extract(p_ref, t1, t2, "median", rows=rows)
            assert np.max(np.abs(host(res[q].C_hat)[rows] - C_ref)) <= tol, q
        else:
            rec = planted_recall(host(res[q].C_hat), w.rows, w.cols, w.tau)
            if rec["recalled"] < rec["planted"]:
                # the estimator itself can miss a planted entry (colliding
                # heavy entries); the oracle's estimate must miss the same ones
                C = O.product(w.A.astype(np.float32).astype(np.float64),
                              w.B.astype(np.float32).astype(np.float64))
                p_ref = O.bucket_sums(C, t1, t2, w.log2b)
                got = host(res[q].C_hat)[w.rows, w.cols]
                ref = np.array([O.extract(p_ref, t1, t2, "median", rows=[i], cols=[j])[0, 0]
                                for i, j in zip(w.rows, w.cols)])
                clear = np.abs(np.abs(ref) - w.tau) > 1e-3 * w.tau
                assert np.array_equal((np.abs(got) >= w.tau)[clear], (np.abs(ref) >= w.tau)[clear]), q
            planted.append(q)
    for q in (min(planted, key=lambda i: ws_list[i].n), max(planted, key=lambda i: ws_list[i].n)):
        w = ws_list[q]
        announce(f"batched mix pair {q} n={w.n} against the oracle")
        t1 = cmm.tables_to_numpy(res[q].tab1)
        t2 = cmm.tables_to_numpy(res[q].tab2)
        C = O.product(w.A, w.B)
        p_ref = O.bucket_sums(C, t1, t2, w.log2b)
        # +-1 operands: their float32 copies are exact
        assert np.max(np.abs(host(res[q].p) - p_ref)) <= f32_tolerance(w.A, w.B, w.log2b, w.n), q
