"""Benchmark: compressed matrix multiplication (FWHT form) on one MI355X.

One step = one full pass of the hot path on resident inputs: hash tables,
A^T copy, bucket plans, fused compress (sketch + WHT + accumulate over k),
partial reduction, inverse WHT (scale 2^-log2b), dense median extract.

Default workload: n = 4096, b = 2^16, d = 9, float64, +-1 entries with
4096 planted pairs A[i] = 4 B[:, j] (synthetic).  The metric is the
DGEMM-equivalent rate 2 n^3 / t, reported with heavy-hitter recall; the
fused compress kernel is reported against the FP64 VALU add roofline, and
the CPU oracle is timed on the host beside it.  The C-ABI steps are also
timed one call at a time (the unfused pipeline) against the HBM roofline.
Beside it: the precision
form (bf16 / fp16 on MFMA, n = 8192), the batched form (64 uneven pairs in
one persistent launch, autotuned, graph replays) and the differentiation
form (forward + adjoint at n = 2048).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz = 39.3e12 adds/s
# (the 78.6 TFLOP/s FP64 vector peak counts an FMA as two flops).
PEAK_F64_ADD = 256 * 4 * 16 * 2.4e9
PEAK_HBM = 8.0e12
PEAK_MFMA_16 = 2.5e15   # dense bf16 / fp16 matrix-core peak
# float32 adds: the published figure (78.6e12/s) counts 2 per lane and cycle,
# which needs packed instructions.  The library is compiled without them, so
# at most half of it (one per lane and cycle) is attainable; fractions are
# still reported against the published figure.
PEAK_F32_ADD = 2 * 256 * 4 * 16 * 2.4e9


# HBM bytes of one float64 compress launch at the default workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) of
#   bench.py --steps 2 --warmup 1 --no-cpu --no-forms --copy-probe 1024
# each scaled by what the same counter reads for the probe's plain 1 GiB
# elementwise copy (fetch x2.000, write x1.000; profiles/
# compress_f64_planted_n4096_b2e16_d9_counters.md).  Reported only while the
# kernel's sources are the ones the counters were taken on.
TRAFFIC_SOURCES = ["paper_2601_09477_amd/csrc/k_compress.hip",
                   "paper_2601_09477_amd/csrc/wht_regs.h",
                   "paper_2601_09477_amd/csrc/api.hip"]   # the launch plan (k-ranges)
TRAFFIC_MEASURED = {"sha1": "b1be4022ffb9552ae96d0b680519634bb51eaf18",
                    "fetch_bytes": 1.1482e+09, "write_bytes": 1.5099e+08}


def compress_traffic():
    """Measured HBM bytes per launch, or None once the kernel has changed."""
    import hashlib
    h = hashlib.sha1()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC_MEASURED["sha1"]:
        return None
    return TRAFFIC_MEASURED["fetch_bytes"] + TRAFFIC_MEASURED["write_bytes"]


def compress_ops(n: int, d: int, log2b: int) -> float:
    """Algorithmic work of Compress (per launch = all k): 2 d n b log2 b
    butterfly adds + 2 d n^2 sketch adds + d n b accumulate FMAs."""
    b = 1 << log2b
    return 2.0 * d * n * b * log2b + 2.0 * d * n * n + 1.0 * d * n * b


def compress_executed_ops(n: int, d: int, log2b: int, log2b_lo: int = 13) -> float:
    """Work the float64 compress kernel executes per launch, in the same units
    as compress_ops.  Each work-group transforms a slice of b_lo = 2^13
    points (log2 b_lo butterfly levels); the b_hi = b / b_lo slices fold the
    top bits into signs, so every slice gathers all n rows of its sketch
    again.  2 d n b log2 b_lo butterfly adds + 2 d n^2 b_hi sketch adds
    (one per gathered row, as compress_ops counts them) + d n b FMAs."""
    b = 1 << log2b
    lo = min(log2b, log2b_lo)
    b_hi = 1 << (log2b - lo)
    return 2.0 * d * n * b * lo + 2.0 * d * n * n * b_hi + 1.0 * d * n * b


def cpu_baseline(w, budget_s: float = 20.0) -> dict:
    """Time the CPU oracle (plain float64 definitions) on the host."""
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:   # threadpoolctl missing: report the process affinity
        blas_threads = len(os.sched_getaffinity(0))
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        t1, t2 = O.hash_tables(w.keys, w.n, w.n, w.log2b)
        C = O.product(w.A, w.B)
        p = O.bucket_sums(C, t1, t2, w.log2b)
        O.extract(p, t1, t2, "median")
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > budget_s * 0.5 or len(times) >= 3:
            break
    t = float(np.median(times))
    return {"value": 2.0 * w.n ** 3 / t / 1e12, "unit": "TFLOP/s-equivalent (2n^3/s)",
            "cores": int(blas_threads), "kind": "oracle",
            "sample": f"full workload (hash + float64 matmul + bucket sums + dense median), "
                      f"{len(times)} run(s), median {t:.2f} s; the matmul uses "
                      f"{blas_threads} BLAS threads, the rest one thread"}


def timed_loop(step, steps: int, dominant: str, kernels, breakdown: int = 3):
    """Time `steps` calls of step() (warm-up done by the caller).  Inside the
    timed region only the launches of `dominant` are bracketed by the
    library's HIP events: each event record delays the stream's next launch
    by a few microseconds, so bracketing every kernel would slow the step
    being timed.  `breakdown` more calls after the timed region, with every
    kernel bracketed, give the other kernels' times.  Returns (ms per step,
    (total ms, launches) of `dominant` in the timed region, {kernel: ms per
    step})."""
    import torch

    import paper_2601_09477_amd as cmm
    cmm.cmm_profile_only(dominant)
    cmm.cmm_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    dom = cmm.cmm_profile_query(dominant)
    cmm.cmm_profile_only(None)
    cmm.cmm_profile_enable(True)
    for _ in range(breakdown):
        step()
    torch.cuda.synchronize()
    per_step = {k: cmm.cmm_profile_query(k)[0] / breakdown for k in kernels}
    per_step[dominant] = dom[0] / steps
    cmm.cmm_profile_enable(False)
    return ms, dom, per_step


def run_estimate(w, compute: str, steps: int, warmup: int, out_dtype=None):
    """Time `steps` full estimates of workload w (inputs resident on the GPU).
    Returns (ms_per_step, (total ms, launches) of the compress in the timed
    region, per-kernel ms per step, C_hat on the GPU, p)."""
    import torch

    import paper_2601_09477_amd as cmm
    n_rows, n_cols = w.A.shape[0], w.B.shape[1]
    d, log2b = w.d, w.log2b
    dev = torch.device("cuda:0")
    A = torch.from_numpy(w.A).to(dev)
    B = torch.from_numpy(w.B).to(dev)
    keys = cmm.keys_tensor(w.keys, dev)
    tab1 = torch.empty((d, n_rows), dtype=torch.int32, device=dev)
    tab2 = torch.empty((d, n_cols), dtype=torch.int32, device=dev)
    p = torch.empty((d, 1 << log2b), dtype=torch.float64, device=dev)
    C_hat = torch.empty((n_rows, n_cols), dtype=out_dtype or torch.float64, device=dev)
    pr = cmm.make_problem(A, B, d, log2b, keys=keys, tab1=tab1, tab2=tab2, p=p, C_hat=C_hat,
                          compute=compute, estimator=w.estimator)
    nbytes = cmm.cmm_workspace_size(pr)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        cmm.cmm_estimate(pr, ws, nbytes, stream)
    torch.cuda.synchronize()
    ms, dom, per_step = timed_loop(
        lambda: cmm.cmm_estimate(pr, ws, nbytes, stream), steps, "compress",
        ("hash", "transpose", "plan", "pairs", "compress", "reduce", "fwht", "extract"))
    del ws
    return ms, dom, per_step, C_hat, p


def heavy_hitter_extract(w, p, steps: int) -> dict:
    """The heavy hitters above tau straight from the sketch p (no dense
    output), timed beside the dense extract of the headline step."""
    import torch

    import paper_2601_09477_amd as cmm
    dev = p.device
    tab1 = torch.empty((w.d, w.n), dtype=torch.int32, device=dev)
    tab2 = torch.empty_like(tab1)
    keys = cmm.keys_tensor(w.keys, dev)
    cmm.cmm_hash(keys, w.d, w.n, w.n, w.log2b, tab1, tab2)
    cap = 1 << 20
    rows = torch.empty(cap, dtype=torch.int64, device=dev)
    cols = torch.empty(cap, dtype=torch.int64, device=dev)
    vals = torch.empty(cap, dtype=torch.float64, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    args = (p, tab1, tab2, w.d, w.n, w.n, w.log2b, cmm.CMM_MEDIAN, w.tau, rows, cols, vals, count)
    cmm.cmm_extract_heavy(*args)
    torch.cuda.synchronize()
    cmm.cmm_profile_enable(True)
    for _ in range(steps):
        cmm.cmm_extract_heavy(*args)
    torch.cuda.synchronize()
    ms, n = cmm.cmm_profile_query("extract_heavy")
    cmm.cmm_profile_enable(False)
    out = {"threshold": w.tau, "hits": int(count.item()), "ms": ms / max(1, n)}
    # the k largest |C_hat| with k = the number of planted entries, sorted,
    # without the dense output or a host synchronisation
    k = len(w.rows)
    trows = torch.empty(k, dtype=torch.int64, device=dev)
    tcols = torch.empty(k, dtype=torch.int64, device=dev)
    tvals = torch.empty(k, dtype=torch.float64, device=dev)
    ws = torch.empty(max(1, cmm.cmm_topk_workspace_size(k)), dtype=torch.uint8, device=dev)
    targs = (p, tab1, tab2, w.d, w.n, w.n, w.log2b, cmm.CMM_MEDIAN, k, trows, tcols, tvals)
    cmm.cmm_extract_topk(*targs, workspace=ws)
    torch.cuda.synchronize()
    cmm.cmm_profile_enable(True)
    for _ in range(steps):
        cmm.cmm_extract_topk(*targs, workspace=ws)
    torch.cuda.synchronize()
    ms, n = cmm.cmm_profile_query("extract_topk")
    cmm.cmm_profile_enable(False)
    got = set(zip(trows.cpu().tolist(), tcols.cpu().tolist()))
    planted = set(zip(np.asarray(w.rows).tolist(), np.asarray(w.cols).tolist()))
    out["topk"] = {"k": k, "ms": ms / max(1, n), "planted_in_topk": len(got & planted),
                   "planted": len(planted)}
    return out


HBM_PEAK_GBS = 8000.0


def unfused_steps(w, steps: int, warmup: int, kc: int = 64) -> dict:
    """The C-ABI steps one call at a time on the headline workload: hash,
    the sketches of A and B for one chunk of kc values of k, their forward
    transforms, the accumulate, the inverse transform and the dense extract.
    Each is reported against the HBM roofline with its algorithmic bytes
    (every input read once, every output written once), and the chunk's
    sketch + transform + accumulate time is scaled to all n values of k to
    set the unfused Compress beside the fused kernel."""
    import torch

    import paper_2601_09477_amd as cmm
    n, d, log2b = w.n, w.d, w.log2b
    b = 1 << log2b
    dev = torch.device("cuda:0")
    A = torch.from_numpy(w.A).to(dev)
    B = torch.from_numpy(w.B).to(dev)
    keys = cmm.keys_tensor(w.keys, dev)
    tab1 = torch.empty((d, n), dtype=torch.int32, device=dev)
    tab2 = torch.empty_like(tab1)
    X = torch.empty((d, kc, b), dtype=torch.float64, device=dev)
    Y = torch.empty_like(X)
    p_hat = torch.zeros((d, b), dtype=torch.float64, device=dev)
    C_hat = torch.empty((n, n), dtype=torch.float64, device=dev)

    def step():
        cmm.cmm_hash(keys, d, n, n, log2b, tab1, tab2)
        cmm.cmm_sketch(0, A, n, n, n, tab1, d, log2b, 0, kc, X)
        cmm.cmm_sketch(1, B, n, n, n, tab2, d, log2b, 0, kc, Y)
        cmm.cmm_fwht(X, d * kc, log2b)
        cmm.cmm_fwht(Y, d * kc, log2b)
        cmm.cmm_accumulate(X, Y, d, kc, log2b, p_hat)
        cmm.cmm_fwht(p_hat, d, log2b, 2.0 ** -log2b)
        cmm.cmm_extract(p_hat, tab1, tab2, d, n, n, log2b, cmm.CMM_MEDIAN, C_hat)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    cmm.cmm_profile_enable(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = {k: cmm.cmm_profile_query(k)[0] / steps
          for k in ("hash", "sketch", "fwht", "accumulate", "extract")}
    cmm.cmm_profile_enable(False)
    vec = d * kc * b * 8                      # one operand's chunk of sketches
    algo = {"hash": 2 * d * n * 4,
            "sketch": 2 * (n * kc * 8 + vec),
            "fwht": 2 * 2 * vec + 2 * d * b * 8,
            "accumulate": 2 * vec + 2 * d * b * 8,
            "extract": n * n * 8 + d * b * 8 + 2 * d * n * 4}
    # a transform of length 2^log2b >= 4096 makes 1 + ceil((log2b - 12) / 4)
    # passes through HBM (12 bits, then 4 at a time)
    passes = 1 + (max(0, log2b - 12) + 3) // 4
    rows = {}
    for k, t in ms.items():
        gbs = algo[k] / (t * 1e-3) / 1e9
        rows[k] = {"ms": t, "algorithmic_bytes": algo[k], "GB_per_s": gbs,
                   "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
    # the extract against the random-gather rate at its footprint: as many
    # gathers (d n^2) as it makes, over a table as long as p
    sink = torch.zeros(1, dtype=torch.float64, device=dev)
    gathers = d * n * n
    cmm.cmm_gather_probe(p_hat, gathers, sink)
    times = []
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        issued = cmm.cmm_gather_probe(p_hat, gathers, sink)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    probe_rate = issued / (sorted(times)[1] * 1e-3)
    extract_rate = gathers / (ms["extract"] * 1e-3)
    rows["extract"].update({"gathers": gathers, "gathers_per_s": extract_rate,
                            "probe_gathers_per_s": probe_rate,
                            "frac_of_probe_gather_rate": extract_rate / probe_rate})
    rows["fwht"]["passes"] = passes
    rows["fwht"]["pass_GB_per_s"] = passes * rows["fwht"]["GB_per_s"]
    rows["fwht"]["pass_frac_of_hbm_peak"] = passes * rows["fwht"]["frac_of_hbm_peak"]
    chunk = ms["sketch"] + ms["fwht"] + ms["accumulate"]
    return {"workload": f"planted +-1, n={n}, b=2^{log2b}, d={d}; one chunk of kc={kc} values of k",
            "kernels": rows,
            "note": "fwht = two forward transforms of d*kc vectors and the inverse of d vectors",
            "unfused_compress_ms_all_k": chunk * n / kc}


def precision_form(steps: int, warmup: int) -> dict:
    """The precision form at n = 8192, b = 2^18, d = 9 (planted +-1, two
    planted columns per row): bf16 and fp16 on MFMA against plain float64 on
    the same GPU (speed, error of p, heavy-hitter recall)."""
    import torch

    from workloads import planted_8192
    from workloads.metrics import planted_recall
    w = planted_8192(0)
    out = {"workload": "planted +-1, n=8192, b=2^18, d=9, 16384 planted pairs (two per row)"}
    ref_p = None
    ref_ms = None
    for compute in ("f64", "bf16", "f16"):
        ms, (ms_c, n_c), _, C_hat, p = run_estimate(w, compute, steps, warmup)
        rec = planted_recall(C_hat.cpu().numpy(), w.rows, w.cols, w.tau)
        avg_c = ms_c / max(1, n_c) * 1e-3
        entry = {"ms_per_step": ms, "value": 2.0 * w.n ** 3 / (ms * 1e-3) / 1e12,
                 "compress_ms": avg_c * 1e3,
                 "recall": {"recalled": rec["recalled"], "planted": rec["planted"],
                            "background_ge_tau": rec["background_ge_tau"]}}
        if compute == "f64":
            ref_p, ref_ms = p, ms
            entry["compress_roofline"] = {
                "bound": "alu", "achieved": compress_ops(w.n, w.d, w.log2b) / avg_c / 1e12,
                "peak": PEAK_F64_ADD / 1e12, "unit": "TFLOP/s",
                "frac": compress_ops(w.n, w.d, w.log2b) / avg_c / PEAK_F64_ADD}
        else:
            dp = (p - ref_p).abs()
            entry["error_vs_f64"] = {"max_abs_dp_over_max_abs_p": float(dp.max() / ref_p.abs().max()),
                                     "rms_dp_over_rms_p": float(dp.pow(2).mean().sqrt() /
                                                                ref_p.pow(2).mean().sqrt())}
            entry["speedup_vs_f64"] = ref_ms / ms
            # executed matrix-core work: 4 passes x 16 MACs x 2 flops per element
            mfma_flops = 2.0 * w.d * w.n * (1 << w.log2b) * 4 * 16 * 2
            entry["compress_roofline"] = {
                "bound": "mfma", "achieved": mfma_flops / avg_c / 1e12, "peak": PEAK_MFMA_16 / 1e12,
                "unit": "TFLOP/s", "frac": mfma_flops / avg_c / PEAK_MFMA_16,
                "algorithmic_add_rate_TFLOPs": compress_ops(w.n, w.d, w.log2b) / avg_c / 1e12}
        out[compute] = entry
        del C_hat, p
        torch.cuda.empty_cache()
    del ref_p
    out["gaussian"] = precision_error_gaussian()
    return out


def precision_error_gaussian() -> dict:
    """The precision form's error on the same shape with N(0,1) entries
    (n = 8192, b = 2^18, d = 9, one planted row per row of A at scale 3):
    on the +-1 inputs bf16 and fp16 are nearly exact, here their rounding
    shows.  One short run per compute type; errors of p and of C_hat against
    the float64 path on the same GPU (itself checked against the float64
    oracle in the test suite)."""
    import torch

    from workloads import planted_8192
    from workloads.metrics import planted_recall
    w = planted_8192(0, gaussian=True)
    out = {"workload": "N(0,1) entries, n=8192, b=2^18, d=9, 8192 planted rows at scale 3"}
    ref_p = ref_C = None
    for compute in ("f64", "bf16", "f16"):
        ms, _, _, C_hat, p = run_estimate(w, compute, 2, 1)
        rec = planted_recall(C_hat.cpu().numpy(), w.rows, w.cols, w.tau)
        entry = {"ms_per_step": ms,
                 "recall": {"recalled": rec["recalled"], "planted": rec["planted"]}}
        if compute == "f64":
            ref_p, ref_C = p, C_hat
        else:
            dp = (p - ref_p).abs()
            dC = (C_hat - ref_C).abs()
            entry["error_vs_f64"] = {
                "max_abs_dp_over_max_abs_p": float(dp.max() / ref_p.abs().max()),
                "rms_dp_over_rms_p": float(dp.pow(2).mean().sqrt() / ref_p.pow(2).mean().sqrt()),
                "max_abs_dC_over_tau": float(dC.max() / w.tau)}
            del C_hat, p
        out[compute] = entry
        torch.cuda.empty_cache()
    return out


def batched_form(steps: int, warmup: int) -> dict:
    """The batched form: 64 pairs, n uniform over {512, 1024, 2048, 4096},
    b = 16 n, d = 7, float32, all Compress work in one persistent launch;
    autotuned, then timed eagerly and as replays of a captured graph."""
    import torch

    import paper_2601_09477_amd as cmm
    from workloads import batched_mix
    from workloads.metrics import planted_recall
    ws_list = batched_mix(0)
    pairs = [(torch.from_numpy(w.A).to("cuda", torch.float32),
              torch.from_numpy(w.B).to("cuda", torch.float32), w.d, w.log2b, w.keys)
             for w in ws_list]
    batch, res = cmm.make_batch(pairs, compute="f32")
    ws = batch.workspace()
    t0 = time.perf_counter()
    cfg = batch.autotune(ws)
    tune_s = time.perf_counter() - t0
    for _ in range(warmup):
        batch.run(ws)
    torch.cuda.synchronize()
    cmm.cmm_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.run(ws)
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) / steps * 1e3
    ms_c, n_c = cmm.cmm_profile_query("compress")
    cmm.cmm_profile_enable(False)
    avg_c = ms_c / max(1, n_c) * 1e-3
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run(ws)
    torch.cuda.current_stream().wait_stream(s)
    with torch.cuda.graph(g):
        batch.run(ws)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) / steps * 1e3
    flops = sum(2.0 * w.n ** 3 for w in ws_list)
    ops = sum(compress_ops(w.n, w.d, w.log2b) for w in ws_list)
    recalled = planted = 0
    for q, w in enumerate(ws_list):
        if w.kind == "planted":
            r = planted_recall(res[q].C_hat.cpu().numpy(), w.rows, w.cols, w.tau)
            recalled += r["recalled"]
            planted += r["planted"]
    out = {"workload": "64 pairs, n in {512,1024,2048,4096} (seed 0), b=16n, d=7, float32; "
                       "32 exactly-sparse Hadamard pairs, 32 planted +-1 pairs",
           "sizes": {str(n): sum(1 for w in ws_list if w.n == n) for n in (512, 1024, 2048, 4096)},
           "config": cfg, "autotune_s": tune_s,
           "ms_per_batch_eager": eager_ms, "ms_per_batch_graph": graph_ms,
           "value": flops / (graph_ms * 1e-3) / 1e12, "unit": "TFLOP/s-equivalent (sum 2n^3/s)",
           "compress_ms": avg_c * 1e3,
           "planted_recall": {"recalled": recalled, "planted": planted},
           "compress_roofline": {
               "bound": "alu", "achieved": ops / avg_c / 1e12, "peak": PEAK_F32_ADD / 1e12,
               "unit": "TFLOP/s", "frac": ops / avg_c / PEAK_F32_ADD,
               "note": "float32 add peak with packed math; 39.3 without"}}
    batch.close()
    del ws, res, pairs
    torch.cuda.empty_cache()
    return out


def differentiation_form(steps: int, warmup: int) -> dict:
    """The differentiation form at n = 2048, b = 2^15, d = 7, float32, mean
    estimator: forward (cmm_estimate) plus the hand-written adjoint
    (cmm_estimate_backward) through the autograd Function."""
    import torch

    import paper_2601_09477_amd as cmm
    from paper_2601_09477_amd.autograd import compressed_matmul
    from workloads import gradient_2048
    w = gradient_2048(0)
    A = torch.from_numpy(w.A).to("cuda", torch.float32).requires_grad_(True)
    B = torch.from_numpy(w.B).to("cuda", torch.float32).requires_grad_(True)
    W = torch.from_numpy(w.W).to("cuda", torch.float32)

    def step():
        A.grad = None
        B.grad = None
        C = compressed_matmul(A, B, w.d, w.log2b, keys=w.keys, compute="f32")
        C.backward(W)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ms, (ms_a, n_a), per_step = timed_loop(
        step, steps, "adjoint",
        ("compress", "extract", "wscatter", "adjoint", "adjoint_reduce", "plan", "transpose",
         "fwht"))
    b = 1 << w.log2b
    n, d = w.n, w.d
    # adjoint: forward transforms again, the transposed transforms (4 d n b log2 b),
    # the products (2 d n b), sketches and transposed sketches (4 d n^2)
    adj_ops = 4.0 * d * n * b * w.log2b + 2.0 * d * n * b + 4.0 * d * n * n
    avg_a = ms_a / max(1, n_a) * 1e-3
    return {"workload": "Gaussian + 2048 planted rows (3x), n=2048, b=2^15, d=7, float32, mean",
            "ms_per_step_fwd_bwd": ms,
            "kernels_ms_per_step": per_step,
            "adjoint_roofline": {"bound": "alu", "achieved": adj_ops / avg_a / 1e12,
                                 "peak": PEAK_F32_ADD / 1e12, "unit": "TFLOP/s",
                                 "frac": adj_ops / avg_a / PEAK_F32_ADD}}


def fft_form(steps: int, warmup: int, seed: int = 0) -> dict:
    """Pagh's FFT form (Section 3.1) on the headline workload (planted +-1,
    n = 4096, b = 2^16, d = 9): the same timed region as the headline
    (hash + compress + inverse + dense extract) through cmm_estimate_fft.
    The paper compares the two transforms on one machine (its SU3 column);
    fwht_speedup is this form's time over the FWHT form's."""
    import torch

    import paper_2601_09477_amd as cmm
    from workloads import planted_4096
    from workloads.metrics import planted_recall
    w = planted_4096(seed)
    dev = torch.device("cuda:0")
    A = torch.from_numpy(w.A).to(dev)
    B = torch.from_numpy(w.B).to(dev)
    keys = cmm.keys_tensor(w.keys, dev)
    d, log2b, n = w.d, w.log2b, w.n
    tab1 = torch.empty((d, n), dtype=torch.int32, device=dev)
    tab2 = torch.empty((d, n), dtype=torch.int32, device=dev)
    p = torch.empty((d, 1 << log2b), dtype=torch.float64, device=dev)
    C_hat = torch.empty((n, n), dtype=torch.float64, device=dev)
    pr = cmm.make_problem(A, B, d, log2b, keys=keys, tab1=tab1, tab2=tab2, p=p, C_hat=C_hat,
                          compute="f64", estimator="median")
    nbytes = cmm.cmm_fft_workspace_size(pr)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        cmm.cmm_estimate_fft(pr, ws, nbytes, stream)
    torch.cuda.synchronize()
    ms, _, per_step = timed_loop(
        lambda: cmm.cmm_estimate_fft(pr, ws, nbytes, stream), steps, "compress",
        ("hash", "sketch", "fft", "accumulate", "compress", "extract"))
    rec = planted_recall(C_hat.cpu().numpy(), w.rows, w.cols, w.tau)
    b = 1 << log2b
    # executed forward transforms of the fused kernel: per (t, slice u_hi <=
    # b_hi / 2, k) two of 4096 points, at 5 N log2 N flops each (the usual
    # count for a radix-2 transform)
    slices = (b >> 12) // 2 + 1
    flops = 2.0 * d * slices * n * 5.0 * 4096 * 12
    comp_ms = per_step["compress"]
    return {"workload": "planted +-1, n=4096, b=2^16, d=9 (the headline), h = h1 + h2 mod b",
            "ms_per_step": ms, "value": 2.0 * n ** 3 / (ms * 1e-3) / 1e12,
            "unit": "TFLOP/s-equivalent (2n^3/s)",
            "kernels_ms_per_step": per_step,
            "compress_transform_rate_TFLOPs": flops / (comp_ms * 1e-3) / 1e12 if comp_ms > 0 else None,
            "recall": {"planted": rec["planted"], "recalled": rec["recalled"]},
            "workspace_bytes": nbytes}


def evaluation_protocol(n_var: int = 1024, draws: int = 1000, n_corr: int = 8192,
                        instances: int = 10, c_d: float = 1.0, c_b: float = 16.0) -> dict:
    """The paper's evaluation protocol on the GPU (Sections 5.2-5.4).

    Variance experiment: per instance family, one instance at n = n_var and
    `draws` independent hash draws (repetition t of one estimate is draw t),
    the single-repetition estimates of the first big entry for several b:
    sample mean and variance against Pagh's bound ||C||_F^2 / b; COVARIANCE
    also under the other two hash families.  Correctness experiment: per
    family `instances` instances at n = n_corr (each with its own hash draw),
    d and b from Section 5.6 with (c_d, c_b), the four counters of Section
    5.4 against the exact product (a float64 GEMM), reported as the columns
    of the paper's correctness table.  Instances are generated on the GPU."""
    import math

    import torch

    import paper_2601_09477_amd as cmm
    from workloads import draw_family_keys, draw_keys
    from workloads import instances as I
    dev = torch.device("cuda:0")
    t_start = time.perf_counter()
    var_rows = []
    for fam in I.FAMILIES:
        w = I.instance(fam, n_var, 100, dev)
        C = w.A @ w.B
        i, j = int(w.big_rows[0]), int(w.big_cols[0])
        cij = float(C[i, j])
        fro2 = float((C * C).sum()) - cij * cij
        ri = torch.tensor([i], dtype=torch.int64, device=dev)
        ci = torch.tensor([j], dtype=torch.int64, device=dev)
        hashes = ["multiply_add_shift"] + (["multiply_shift", "tabulation"]
                                           if fam == "covariance" else [])
        for h in hashes:
            for log2b in (10, 12, 14, 16):
                keys = draw_family_keys(h, draws, 31337 + log2b)
                tab1, tab2 = cmm.family_tables(h, keys, n_var, n_var, log2b, dev)
                res = cmm.estimate(w.A, w.B, draws, log2b, tab1=tab1, tab2=tab2,
                                   estimator="mean", dense=False)
                x = torch.empty((draws, 1), dtype=torch.float64, device=dev)
                cmm.cmm_extract_reps(res.p, tab1, tab2, draws, n_var, n_var, log2b, ri, ci, x)
                xs = x[:, 0].double()
                var = float(xs.var(unbiased=True))
                var_rows.append({"instance": fam, "hash": h, "log2b": log2b, "c": cij,
                                 "mean": float(xs.mean()), "var": var,
                                 "bound": fro2 / (1 << log2b),
                                 "var_over_bound": var / (fro2 / (1 << log2b))})
        del w, C
    t_var = time.perf_counter() - t_start
    print(f"[bench] variance experiment {t_var:.1f} s", file=sys.stderr, flush=True)

    d, log2b = I.params(n_corr, c_d, c_b)
    corr = {}
    t1 = time.perf_counter()
    for fam in I.FAMILIES:
        fr = {"all_eps": 0.0, "big_eps": 0.0, "big_ge": 0.0, "small_le": 0.0}
        est_ms = 0.0
        for r in range(instances):
            w = I.instance(fam, n_corr, 1000 + r, dev)
            C = w.A @ w.B
            keys = draw_keys(d, 5000 + 97 * r + I.FAMILIES.index(fam))
            torch.cuda.synchronize()
            e0 = time.perf_counter()
            res = cmm.estimate(w.A, w.B, d, log2b, keys=keys)
            torch.cuda.synchronize()
            est_ms += (time.perf_counter() - e0) * 1e3
            counts = torch.empty(4, dtype=torch.int64, device=dev)
            cmm.cmm_correctness_counts(res.C_hat, C, w.big_rows.to(torch.int64),
                                       w.big_cols.to(torch.int64), counts, 0.5, 0.1)
            bge, sle, beps, seps = (int(v) for v in counts.cpu())
            nb = int(w.big_rows.numel())
            ns = n_corr * n_corr - nb
            fr["all_eps"] += (beps + seps) / (n_corr * n_corr) / instances
            fr["big_eps"] += beps / nb / instances
            fr["big_ge"] += bge / nb / instances
            fr["small_le"] += sle / ns / instances
            del w, C, res
        fr["ms_per_estimate"] = est_ms / instances
        corr[fam] = fr
        print(f"[bench] correctness {fam} done", file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    return {"variance": {"n": n_var, "draws": draws, "rows": var_rows, "seconds": t_var},
            "correctness": {"n": n_corr, "instances": instances, "d": d, "b": 1 << log2b,
                            "c_d": c_d, "c_b": c_b, "threshold": 0.5, "tolerance": 0.1,
                            "families": corr, "seconds": time.perf_counter() - t1}}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision-form leg")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-eval", action="store_true",
                    help="skip the evaluation protocol (variance and correctness experiments)")
    ap.add_argument("--only-precision", action="store_true",
                    help="run only the precision-form leg and print it (for counter runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run one plain elementwise copy of MIB MiB (read MIB, write "
                         "MIB): the reference dispatch for hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the path runs on one GPU; sharding over several is a design note only)", file=sys.stderr)
        return 2
    if args.only_precision:
        # the precision form's leg alone (for hardware-counter runs of its kernels)
        print(json.dumps({"mfma_form": precision_form(max(3, args.steps // 4), 1)}), flush=True)
        return 0

    from workloads import planted_4096
    from workloads.metrics import planted_recall

    if args.copy_probe > 0:
        import torch
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    w = planted_4096(args.seed)
    n, d, log2b = w.n, w.d, w.log2b
    ms_per_step, (ms_comp, n_comp), per_step, C_hat, p = run_estimate(w, "f64", args.steps,
                                                                       args.warmup)
    rec = planted_recall(C_hat.cpu().numpy(), w.rows, w.cols, w.tau)
    heavy = heavy_hitter_extract(w, p, args.steps)
    unfused = unfused_steps(w, max(3, args.steps // 2), 1)
    avg_comp = ms_comp / max(1, n_comp) * 1e-3
    ops = compress_ops(n, d, log2b)
    achieved = ops / avg_comp
    executed = compress_executed_ops(n, d, log2b)
    out = {
        "metric": "effective 2n^3/s + heavy-hitter recall, plain FP64 vs MFMA form, 1 GPU",
        "value": 2.0 * n ** 3 / (ms_per_step * 1e-3) / 1e12,
        "unit": "TFLOP/s-equivalent (2n^3/s)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "planted +-1, n=4096, b=2^16, d=9, 4096 planted pairs at 4n",
                   "n": n, "b": 1 << log2b, "d": d, "estimator": "median", "seed": args.seed},
        "recall": {"planted": rec["planted"], "recalled": rec["recalled"],
                   "recall": rec["recall"], "background_ge_tau": rec["background_ge_tau"],
                   "tau": w.tau},
        "kernels_ms_per_step": per_step,
        "heavy_hitter_extract": heavy,
        "unfused_steps": unfused,
        "roofline": {"kernel": "compress (fused sketch + WHT + accumulate)", "bound": "alu",
                     "achieved": achieved / 1e12, "peak": PEAK_F64_ADD / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_F64_ADD,
                     "work_per_launch": ops, "avg_launch_ms": avg_comp * 1e3,
                     "executed_work_per_launch": executed,
                     "executed_TFLOPs": executed / avg_comp / 1e12,
                     "executed_frac": executed / avg_comp / PEAK_F64_ADD,
                     "traffic": compress_traffic()},
    }
    del C_hat
    if not args.no_forms:
        out["mfma_form"] = precision_form(max(3, args.steps // 4), 1)
        out["batched_form"] = batched_form(max(3, args.steps // 4), 1)
        out["differentiation_form"] = differentiation_form(max(3, args.steps // 2), 2)
        out["fft_form"] = fft_form(max(2, args.steps // 10), 1, args.seed)
        out["fft_form"]["fwht_speedup"] = out["fft_form"]["ms_per_step"] / ms_per_step
    if not args.no_eval and not args.no_forms:
        out["evaluation"] = evaluation_protocol()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
