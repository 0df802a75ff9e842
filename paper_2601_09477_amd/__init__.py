"""MI355X (gfx950) compressed matrix multiplication in the FWHT form.

A thin ctypes binding over ``libcmm.so`` (the HIP library declared in
``include/cmm.h``).  The functions named ``cmm_*`` take torch tensors that
live on the GPU and marshal their device pointers and the current HIP
stream into the C ABI of the same name; every step runs in the library's
kernels.  ``estimate`` is the end-to-end convenience wrapper (it allocates
outputs and the workspace with torch).

The library must be built (``python -m paper_2601_09477_amd.build`` or
``__graft_entry__.build()``); importing works without it, but any call
raises ``CmmError`` when ``libcmm.so`` is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcmm.so")

CMM_OK, CMM_EINVAL, CMM_ENOMEM, CMM_EHIP, CMM_EUNSUPPORTED = range(5)
CMM_F64, CMM_F32, CMM_BF16, CMM_F16 = range(4)
CMM_MEDIAN, CMM_MEAN = range(2)
CMM_HASH_MULTIPLY_ADD_SHIFT, CMM_HASH_MULTIPLY_SHIFT, CMM_HASH_TABULATION = range(3)
HASH_FAMILIES = {"multiply_add_shift": CMM_HASH_MULTIPLY_ADD_SHIFT,
                 "multiply_shift": CMM_HASH_MULTIPLY_SHIFT, "tabulation": CMM_HASH_TABULATION}

EXPORTED = ["cmm_hash", "cmm_hash_family", "cmm_sketch", "cmm_fwht", "cmm_accumulate", "cmm_extract",
            "cmm_extract_entries", "cmm_extract_heavy", "cmm_topk_workspace_size",
            "cmm_extract_topk", "cmm_extract_reps",
            "cmm_correctness_counts", "cmm_fft", "cmm_extract_cyclic", "cmm_fft_workspace_size",
            "cmm_estimate_fft",
            "cmm_workspace_size", "cmm_estimate", "cmm_estimate_static",
            "cmm_backward_workspace_size",
            "cmm_estimate_backward", "cmm_batch_create", "cmm_batch_destroy",
            "cmm_batch_workspace_size", "cmm_batch_autotune", "cmm_batch_set_config",
            "cmm_batch_get_config", "cmm_estimate_batched", "cmm_status_string", "cmm_last_error",
            "cmm_abi_version", "cmm_profile_enable", "cmm_profile_only",
            "cmm_profile_query", "cmm_gather_probe"]


class CmmError(RuntimeError):
    """A non-OK status returned by libcmm (or the library is missing)."""

    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_STATUS_NAMES = {0: "CMM_OK", 1: "CMM_EINVAL", 2: "CMM_ENOMEM", 3: "CMM_EHIP",
                 4: "CMM_EUNSUPPORTED"}


class Problem(ctypes.Structure):
    """Mirror of ``cmm_problem`` in include/cmm.h."""
    _fields_ = [("n_rows", ctypes.c_int64), ("n_inner", ctypes.c_int64),
                ("n_cols", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("in_dtype", ctypes.c_int), ("compute", ctypes.c_int),
                ("d", ctypes.c_int), ("log2b", ctypes.c_int), ("estimator", ctypes.c_int),
                ("keys", ctypes.c_void_p), ("tab1", ctypes.c_void_p), ("tab2", ctypes.c_void_p),
                ("p", ctypes.c_void_p),
                ("C_hat", ctypes.c_void_p), ("out_dtype", ctypes.c_int), ("ldc", ctypes.c_int64)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libcmm.so (once) and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise CmmError("load", CMM_EUNSUPPORTED,
                       f"{LIB_PATH} is not built; run python -m paper_2601_09477_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    sig = {
        "cmm_hash": [vp, i32, i64, i64, i32, vp, vp, vp],
        "cmm_hash_family": [i32, vp, i32, i64, i64, i32, vp, vp, vp],
        "cmm_sketch": [i32, vp, i32, i64, i64, i64, vp, i32, i32, i64, i64, vp, i32, vp],
        "cmm_fwht": [vp, i32, i64, i32, dbl, vp],
        "cmm_accumulate": [vp, vp, i32, i32, i64, i32, vp, vp],
        "cmm_extract": [vp, vp, vp, i32, i64, i64, i32, i32, vp, i32, i64, vp],
        "cmm_extract_entries": [vp, vp, vp, i32, i64, i64, i32, i32, vp, vp, i64, vp, i32, vp],
        "cmm_extract_heavy": [vp, vp, vp, i32, i64, i64, i32, i32, dbl, vp, vp, vp, i32, i64, vp,
                              vp],
        "cmm_extract_reps": [vp, vp, vp, i32, i64, i64, i32, vp, vp, i64, vp, i32, vp],
        "cmm_topk_workspace_size": [i64, ctypes.POINTER(ctypes.c_size_t)],
        "cmm_extract_topk": [vp, vp, vp, i32, i64, i64, i32, i32, i64, vp, vp, vp, i32, vp,
                             ctypes.c_size_t, vp],
        "cmm_fft": [vp, vp, i64, i32, i32, dbl, vp],
        "cmm_extract_cyclic": [vp, vp, vp, i32, i64, i64, i32, i32, vp, i32, i64, vp],
        "cmm_fft_workspace_size": [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t)],
        "cmm_estimate_fft": [ctypes.POINTER(Problem), vp, ctypes.c_size_t, vp],
        "cmm_correctness_counts": [vp, i32, i64, vp, i64, i64, i64, vp, vp, i64, dbl, dbl, vp, vp],
        "cmm_workspace_size": [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t)],
        "cmm_estimate": [ctypes.POINTER(Problem), vp, ctypes.c_size_t, vp],
        "cmm_estimate_static": [ctypes.POINTER(Problem), vp],
        "cmm_backward_workspace_size": [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t)],
        "cmm_estimate_backward": [ctypes.POINTER(Problem), vp, i64, vp, i64, vp, i64, vp,
                                  ctypes.c_size_t, vp],
    }
    sig.update({
        "cmm_batch_create": [ctypes.POINTER(Problem), i32, ctypes.POINTER(vp)],
        "cmm_batch_destroy": [vp],
        "cmm_batch_workspace_size": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "cmm_batch_autotune": [vp, vp, ctypes.c_size_t, vp],
        "cmm_batch_set_config": [vp, i32, i32, i32, i32, i32],
        "cmm_batch_get_config": [vp] + [ctypes.POINTER(i32)] * 6,
        "cmm_estimate_batched": [vp, vp, ctypes.c_size_t, vp],
    })
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.cmm_status_string.argtypes = [ctypes.c_int]
    L.cmm_status_string.restype = ctypes.c_char_p
    L.cmm_last_error.argtypes = []
    L.cmm_last_error.restype = ctypes.c_char_p
    L.cmm_abi_version.argtypes = []
    L.cmm_abi_version.restype = ctypes.c_int
    L.cmm_profile_enable.argtypes = [ctypes.c_int]
    L.cmm_profile_enable.restype = None
    L.cmm_gather_probe.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_uint32, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]
    L.cmm_gather_probe.restype = ctypes.c_int
    L.cmm_profile_only.argtypes = [ctypes.c_char_p]
    L.cmm_profile_only.restype = ctypes.c_int
    L.cmm_profile_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int)]
    L.cmm_profile_query.restype = ctypes.c_int
    _lib = L
    return L


def _check(fn: str, status: int) -> None:
    if status != CMM_OK:
        raise CmmError(fn, status, lib().cmm_last_error().decode())


# ------------------------------------------------------------ marshalling
def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return CMM_F64
    if t.dtype == torch.float32:
        return CMM_F32
    raise CmmError("dtype", CMM_EINVAL, f"unsupported tensor dtype {t.dtype}")


def _ptr(t, ld: bool = False) -> Optional[int]:
    """Device address of t.  The library reads and writes dense row-major
    extents from its size arguments: a buffer must be contiguous, and a
    matrix passed with a leading dimension (ld=True) needs unit stride along
    its rows and no zero strides (an expanded view covers less memory than
    the library would touch)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise CmmError("marshal", CMM_EINVAL, "tensors must live on the GPU")
    if ld:
        if t.dim() == 2 and t.numel() > 0 and (
                (t.shape[1] > 1 and t.stride(1) != 1) or (t.shape[0] > 1 and t.stride(0) < t.shape[1])):
            raise CmmError("marshal", CMM_EINVAL,
                           "a matrix needs unit stride along its rows and a leading dimension "
                           ">= its row length")
    elif not t.is_contiguous():
        raise CmmError("marshal", CMM_EINVAL, "buffers must be contiguous")
    return t.data_ptr()


def _need(ok: bool, fn: str, msg: str) -> None:
    """Raise CmmError(fn, CMM_EINVAL) before any launch unless ok."""
    if not ok:
        raise CmmError(fn, CMM_EINVAL, msg)


def _like(t, fn: str, name: str, dtypes=None, shape=None, min_numel=None) -> None:
    """t is a tensor of one of dtypes (torch dtypes), of exactly shape (a
    tuple) or holding at least min_numel elements: the sizes the library
    will read or write through t's pointer."""
    _need(t is not None, fn, f"{name} is missing")
    if dtypes is not None:
        _need(t.dtype in dtypes, fn, f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if shape is not None:
        _need(tuple(t.shape) == tuple(shape), fn,
              f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if min_numel is not None:
        _need(t.numel() >= min_numel, fn,
              f"{name} holds {t.numel()} elements, the call addresses {min_numel}")


def _floats():
    torch = _torch()
    return (torch.float64, torch.float32)


def _tables(fn, tab1, tab2, d, n_rows, n_cols) -> None:
    i32 = (_torch().int32,)
    if n_rows > 0:
        _like(tab1, fn, "tab1", i32, (d, n_rows))
    if n_cols > 0:
        _like(tab2, fn, "tab2", i32, (d, n_cols))


def _sketch_p(fn, p, d, log2b) -> None:
    _like(p, fn, "p", (_torch().float64,), (d, 1 << log2b))


def _stream(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# -------------------------------------------------------- C-ABI wrappers
def cmm_hash(keys, d, n_rows, n_cols, log2b, tab1, tab2, stream=None) -> None:
    """keys int64[d][4][2] (uint64 bits), tab1 int32[d][n_rows], tab2 int32[d][n_cols]."""
    _like(keys, "cmm_hash", "keys", (_torch().int64,), min_numel=8 * d)
    _tables("cmm_hash", tab1, tab2, d, n_rows, n_cols)
    _check("cmm_hash", lib().cmm_hash(_ptr(keys), d, n_rows, n_cols, log2b, _ptr(tab1),
                                      _ptr(tab2), _stream(stream)))


def cmm_sketch(side, M, rows, cols, ld=None, tab=None, d=None, log2b=None, k0=0, kc=None,
               out=None, stream=None) -> None:
    """Count sketches of columns k0 .. k0 + kc - 1 of A (side 0, M = A) or
    rows of B (side 1, M = B) into out [d][kc][2^log2b] (float64 or float32,
    either input type); ld defaults to M's row stride and must equal it when
    given."""
    fn = "cmm_sketch"
    _like(M, fn, "M", _floats(), (rows, cols))
    ld = M.stride(0) if ld is None else ld
    _need(rows <= 1 or ld == M.stride(0), fn, f"ld {ld} differs from M's row stride {M.stride(0)}")
    _like(tab, fn, "tab", (_torch().int32,), (d, rows if side == 0 else cols))
    _like(out, fn, "out", _floats(), min_numel=d * kc << log2b)
    _check("cmm_sketch", lib().cmm_sketch(side, _ptr(M, True), _dtype_code(M), rows, cols, ld,
                                          _ptr(tab), d, log2b, k0, kc, _ptr(out),
                                          _dtype_code(out), _stream(stream)))


def cmm_fwht(x, batch, log2b, scale=1.0, stream=None) -> None:
    _like(x, "cmm_fwht", "x", _floats(), min_numel=batch << log2b)
    _check("cmm_fwht", lib().cmm_fwht(_ptr(x), _dtype_code(x), batch, log2b, float(scale),
                                      _stream(stream)))


def cmm_accumulate(X, Y, d, kc, log2b, p_hat, stream=None) -> None:
    fn = "cmm_accumulate"
    _like(X, fn, "X", _floats(), min_numel=d * kc << log2b)
    _like(Y, fn, "Y", (X.dtype,), min_numel=d * kc << log2b)
    _like(p_hat, fn, "p_hat", (_torch().float64,), min_numel=d << log2b)
    _check("cmm_accumulate", lib().cmm_accumulate(_ptr(X), _ptr(Y), _dtype_code(X), d, kc,
                                                  log2b, _ptr(p_hat), _stream(stream)))


def cmm_extract(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, C_hat, ldc=None,
                stream=None) -> None:
    fn = "cmm_extract"
    _sketch_p(fn, p, d, log2b)
    _tables(fn, tab1, tab2, d, n_rows, n_cols)
    _like(C_hat, fn, "C_hat", _floats(), (n_rows, n_cols))
    ldc = C_hat.stride(0) if ldc is None else ldc
    _need(n_rows <= 1 or ldc == C_hat.stride(0), fn,
          f"ldc {ldc} differs from C_hat's row stride {C_hat.stride(0)}")
    _check("cmm_extract", lib().cmm_extract(_ptr(p), _ptr(tab1), _ptr(tab2), d, n_rows, n_cols,
                                            log2b, estimator, _ptr(C_hat, True), _dtype_code(C_hat),
                                            ldc, _stream(stream)))


def cmm_extract_entries(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, rows, cols, out,
                        stream=None) -> None:
    """out[q] = estimate at (rows[q], cols[q]); rows, cols int64 device tensors."""
    fn = "cmm_extract_entries"
    _sketch_p(fn, p, d, log2b)
    _tables(fn, tab1, tab2, d, n_rows, n_cols)
    _like(rows, fn, "rows", (_torch().int64,))
    _like(cols, fn, "cols", (_torch().int64,), min_numel=rows.numel())
    _like(out, fn, "out", _floats(), min_numel=rows.numel())
    _check("cmm_extract_entries", lib().cmm_extract_entries(
        _ptr(p), _ptr(tab1), _ptr(tab2), d, n_rows, n_cols, log2b, estimator, _ptr(rows),
        _ptr(cols), rows.numel(), _ptr(out), _dtype_code(out), _stream(stream)))


def cmm_topk_workspace_size(k: int) -> int:
    n = ctypes.c_size_t(0)
    _check("cmm_topk_workspace_size", lib().cmm_topk_workspace_size(k, ctypes.byref(n)))
    return n.value


def cmm_extract_topk(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, k, rows, cols, vals,
                     workspace=None, stream=None) -> None:
    """The k entries of largest |C_hat| (sorted by magnitude, ties by the
    smaller row-major index) into rows, cols (int64 [k]) and vals (float64 or
    float32 [k]); workspace: uint8 device tensor of cmm_topk_workspace_size(k)
    bytes (allocated here when None)."""
    fn = "cmm_extract_topk"
    torch = _torch()
    _sketch_p(fn, p, d, log2b)
    _tables(fn, tab1, tab2, d, n_rows, n_cols)
    _like(rows, fn, "rows", (torch.int64,), min_numel=k)
    _like(cols, fn, "cols", (torch.int64,), min_numel=k)
    _like(vals, fn, "vals", _floats(), min_numel=k)
    nbytes = cmm_topk_workspace_size(k)
    if workspace is None:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=p.device)
    _like(workspace, fn, "workspace", (torch.uint8,), min_numel=nbytes)
    _check(fn, lib().cmm_extract_topk(_ptr(p), _ptr(tab1), _ptr(tab2), d, n_rows, n_cols, log2b,
                                      estimator, k, _ptr(rows), _ptr(cols), _ptr(vals),
                                      _dtype_code(vals), _ptr(workspace), workspace.numel(),
                                      _stream(stream)))


def topk(res, n_rows: int, n_cols: int, k: int, estimator: str = "median", dtype=None):
    """Top-k entries of an ``Estimate`` (its p and tables): (rows, cols, vals)."""
    torch = _torch()
    d, b = res.p.shape
    log2b = int(b).bit_length() - 1
    rows = torch.empty(k, dtype=torch.int64, device=res.p.device)
    cols = torch.empty(k, dtype=torch.int64, device=res.p.device)
    vals = torch.empty(k, dtype=dtype or torch.float64, device=res.p.device)
    est = CMM_MEDIAN if estimator == "median" else CMM_MEAN
    cmm_extract_topk(res.p, res.tab1, res.tab2, d, n_rows, n_cols, log2b, est, k, rows, cols, vals)
    return rows, cols, vals


def cmm_extract_reps(p, tab1, tab2, d, n_rows, n_cols, log2b, rows, cols, out,
                     stream=None) -> None:
    """out[t][q] = the repetition-t estimate at (rows[q], cols[q]); out is a
    [d][count] float64 or float32 device tensor."""
    fn = "cmm_extract_reps"
    _sketch_p(fn, p, d, log2b)
    _tables(fn, tab1, tab2, d, n_rows, n_cols)
    _like(rows, fn, "rows", (_torch().int64,))
    _like(cols, fn, "cols", (_torch().int64,), min_numel=rows.numel())
    _like(out, fn, "out", _floats(), min_numel=d * rows.numel())
    _check("cmm_extract_reps", lib().cmm_extract_reps(
        _ptr(p), _ptr(tab1), _ptr(tab2), d, n_rows, n_cols, log2b, _ptr(rows), _ptr(cols),
        rows.numel(), _ptr(out), _dtype_code(out), _stream(stream)))


def cmm_correctness_counts(C_hat, C, big_rows, big_cols, counts, threshold=0.5, tolerance=0.1,
                           stream=None) -> None:
    """Section 5.4 counters into counts (int64 device tensor of 4):
    [big >= thr, small <= thr, big within tol, small within tol]."""
    fn = "cmm_correctness_counts"
    n_rows, n_cols = C_hat.shape
    _like(C_hat, fn, "C_hat", _floats())
    _like(C, fn, "C", (_torch().float64,), (n_rows, n_cols))
    _like(big_rows, fn, "big_rows", (_torch().int64,))
    _like(big_cols, fn, "big_cols", (_torch().int64,), min_numel=big_rows.numel())
    _like(counts, fn, "counts", (_torch().int64,), min_numel=4)
    _check("cmm_correctness_counts", lib().cmm_correctness_counts(
        _ptr(C_hat, True), _dtype_code(C_hat), C_hat.stride(0), _ptr(C, True), C.stride(0), n_rows, n_cols,
        _ptr(big_rows), _ptr(big_cols), big_rows.numel(), threshold, tolerance, _ptr(counts),
        _stream(stream)))


def cmm_extract_heavy(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, threshold, out_rows,
                      out_cols, out_vals, count, stream=None) -> None:
    """Entries with |C_hat| >= threshold into the lists (capacity = their length);
    count: int64 device tensor of one element, receives the number of hits."""
    fn = "cmm_extract_heavy"
    i64 = (_torch().int64,)
    _sketch_p(fn, p, d, log2b)
    _tables(fn, tab1, tab2, d, n_rows, n_cols)
    _like(out_rows, fn, "out_rows", i64)
    _like(out_cols, fn, "out_cols", i64, min_numel=out_rows.numel())
    _like(out_vals, fn, "out_vals", _floats(), min_numel=out_rows.numel())
    _like(count, fn, "count", i64, min_numel=1)
    _check("cmm_extract_heavy", lib().cmm_extract_heavy(
        _ptr(p), _ptr(tab1), _ptr(tab2), d, n_rows, n_cols, log2b, estimator, float(threshold),
        _ptr(out_rows), _ptr(out_cols), _ptr(out_vals), _dtype_code(out_vals), out_rows.numel(),
        _ptr(count), _stream(stream)))


def heavy_hitters(est: "Estimate", threshold: float, capacity: int = 1 << 20,
                  estimator: str = "median", out_dtype=None):
    """(rows, cols, values) of every entry with |C_hat| >= threshold of an
    estimate made with dense=False, sorted by (row, column)."""
    torch = _torch()
    dev = est.p.device
    d, b = est.p.shape
    n_rows, n_cols = est.tab1.shape[1], est.tab2.shape[1]
    rows = torch.empty(capacity, dtype=torch.int64, device=dev)
    cols = torch.empty(capacity, dtype=torch.int64, device=dev)
    vals = torch.empty(capacity, dtype=out_dtype or torch.float64, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    est_code = CMM_MEDIAN if estimator == "median" else CMM_MEAN
    cmm_extract_heavy(est.p, est.tab1, est.tab2, d, n_rows, n_cols, int(b).bit_length() - 1,
                      est_code, threshold, rows, cols, vals, count)
    k = int(count.item())
    if k > capacity:
        raise CmmError("heavy_hitters", CMM_ENOMEM, f"{k} hits exceed capacity {capacity}")
    order = torch.argsort(rows[:k] * n_cols + cols[:k])
    return rows[:k][order], cols[:k][order], vals[:k][order]


def cmm_workspace_size(prob: Problem) -> int:
    n = ctypes.c_size_t(0)
    _check("cmm_workspace_size", lib().cmm_workspace_size(ctypes.byref(prob), ctypes.byref(n)))
    return n.value


def cmm_estimate(prob: Problem, workspace, workspace_bytes: int, stream=None) -> None:
    _check("cmm_estimate", lib().cmm_estimate(ctypes.byref(prob), _ptr(workspace),
                                              workspace_bytes, _stream(stream)))


def cmm_estimate_static(prob: Problem, stream=None) -> None:
    """cmm_estimate with the library's static scratch instead of a workspace
    (allocates nothing; problems up to CMM_STATIC_SCRATCH_BYTES of scratch)."""
    _check("cmm_estimate_static", lib().cmm_estimate_static(ctypes.byref(prob), _stream(stream)))


def cmm_fft_workspace_size(prob: Problem) -> int:
    n = ctypes.c_size_t(0)
    _check("cmm_fft_workspace_size",
           lib().cmm_fft_workspace_size(ctypes.byref(prob), ctypes.byref(n)))
    return n.value


def cmm_estimate_fft(prob: Problem, workspace, workspace_bytes: int, stream=None) -> None:
    _check("cmm_estimate_fft", lib().cmm_estimate_fft(ctypes.byref(prob), _ptr(workspace),
                                                      workspace_bytes, _stream(stream)))


def cmm_fft(x, out, inverse=False, scale=1.0, stream=None) -> None:
    """Batched complex transform along the last axis of complex128 tensors
    (length a power of two); out may be x when the length is <= 4096."""
    torch = _torch()
    n = x.shape[-1]
    _like(x, "cmm_fft", "x", (torch.complex128,))
    _like(out, "cmm_fft", "out", (torch.complex128,), tuple(x.shape))
    _need(n > 0 and n & (n - 1) == 0, "cmm_fft", f"length {n} is not a power of two")
    log2n = n.bit_length() - 1
    batch = x.numel() // n if n else 0
    _check("cmm_fft", lib().cmm_fft(_ptr(x), _ptr(out), batch, log2n, int(bool(inverse)),
                                    float(scale), _stream(stream)))


def cmm_extract_cyclic(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, C_hat,
                       stream=None) -> None:
    fn = "cmm_extract_cyclic"
    _sketch_p(fn, p, d, log2b)
    _tables(fn, tab1, tab2, d, n_rows, n_cols)
    _like(C_hat, fn, "C_hat", _floats(), (n_rows, n_cols))
    _check("cmm_extract_cyclic", lib().cmm_extract_cyclic(
        _ptr(p), _ptr(tab1), _ptr(tab2), d, n_rows, n_cols, log2b, estimator, _ptr(C_hat, True),
        _dtype_code(C_hat), C_hat.stride(0), _stream(stream)))


def estimate_fft(A, B, d: int, log2b: int, *, keys=None, tab1=None, tab2=None,
                 estimator: str = "median", dense: bool = True, workspace=None,
                 stream=None) -> "Estimate":
    """Pagh's FFT form of the compressed product (float64 only)."""
    torch = _torch()
    dev = A.device
    n_rows, n_cols = A.shape[0], B.shape[1]
    if keys is not None and not hasattr(keys, "data_ptr"):
        keys = keys_tensor(keys, dev)
    if keys is not None:
        tab1 = torch.empty((d, n_rows), dtype=torch.int32, device=dev)
        tab2 = torch.empty((d, n_cols), dtype=torch.int32, device=dev)
    p = torch.empty((d, 1 << log2b), dtype=torch.float64, device=dev)
    C_hat = torch.empty((n_rows, n_cols), dtype=torch.float64, device=dev) if dense else None
    pr = make_problem(A, B, d, log2b, keys=keys, tab1=tab1, tab2=tab2, p=p, C_hat=C_hat,
                      compute="f64", estimator=estimator)
    nbytes = cmm_fft_workspace_size(pr)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    cmm_estimate_fft(pr, workspace, nbytes, stream)
    return Estimate(C_hat, p, tab1, tab2)


def cmm_backward_workspace_size(prob: Problem) -> int:
    n = ctypes.c_size_t(0)
    _check("cmm_backward_workspace_size",
           lib().cmm_backward_workspace_size(ctypes.byref(prob), ctypes.byref(n)))
    return n.value


def cmm_estimate_backward(prob: Problem, W, dA, dB, workspace, workspace_bytes: int,
                          stream=None) -> None:
    """dA, dB of L = sum(W o C_hat) for the mean-over-d estimate of ``prob``."""
    fn = "cmm_estimate_backward"
    dt = (prob._tensors[0].dtype,)
    _like(W, fn, "W", dt, (prob.n_rows, prob.n_cols))
    _like(dA, fn, "dA", dt, (prob.n_rows, prob.n_inner))
    _like(dB, fn, "dB", dt, (prob.n_inner, prob.n_cols))
    _check("cmm_estimate_backward",
           lib().cmm_estimate_backward(ctypes.byref(prob), _ptr(W, True), W.stride(0), _ptr(dA, True),
                                       dA.stride(0), _ptr(dB, True), dB.stride(0), _ptr(workspace),
                                       workspace_bytes, _stream(stream)))


def cmm_profile_enable(on: bool = True) -> None:
    lib().cmm_profile_enable(1 if on else 0)


def cmm_gather_probe(table, gathers: int, sink, seed: int = 0, stream=None) -> int:
    """Random 8-byte gathers from a float64 CUDA tensor (a measurement aid);
    returns the number issued."""
    if table.dtype != _torch().float64 or sink.dtype != _torch().float64:
        raise TypeError("cmm_gather_probe: table and sink must be float64")
    if not table.is_contiguous():
        raise ValueError("cmm_gather_probe: the table must be contiguous (its numel is the length)")
    issued = ctypes.c_int64(0)
    _check("cmm_gather_probe",
           lib().cmm_gather_probe(_ptr(table), table.numel(), int(gathers), seed & 0xFFFFFFFF,
                                  _ptr(sink), ctypes.byref(issued), _stream(stream)))
    return issued.value


def cmm_profile_only(kernel=None) -> None:
    """Bracket only the launches of one kernel with timing events (None: all)."""
    _check("cmm_profile_only", lib().cmm_profile_only(kernel.encode() if kernel else None))


def cmm_profile_query(kernel: str):
    """(total milliseconds, launches) of one kernel since profiling was enabled."""
    ms, n = ctypes.c_double(0.0), ctypes.c_int(0)
    _check("cmm_profile_query", lib().cmm_profile_query(kernel.encode(), ctypes.byref(ms),
                                                        ctypes.byref(n)))
    return ms.value, n.value


# ------------------------------------------------------------ high level
_COMPUTE = {"f64": CMM_F64, "f32": CMM_F32, "bf16": CMM_BF16, "f16": CMM_F16}


def cmm_hash_family(kind, keys, d, n_rows, n_cols, log2b, tab1, tab2, stream=None) -> None:
    """kind CMM_HASH_*; keys int64 [d][4][2] (multiply families) or [d][4][4][256]
    (tabulation), uint64 bits; tables as for cmm_hash."""
    fn = "cmm_hash_family"
    per_t = 4 * 4 * 256 if kind == CMM_HASH_TABULATION else 8
    _like(keys, fn, "keys", (_torch().int64,), min_numel=per_t * d)
    _tables(fn, tab1, tab2, d, n_rows, n_cols)
    _check("cmm_hash_family", lib().cmm_hash_family(kind, _ptr(keys), d, n_rows, n_cols, log2b,
                                                    _ptr(tab1), _ptr(tab2), _stream(stream)))


def family_tables(family: str, keys: np.ndarray, n_rows: int, n_cols: int, log2b: int,
                  device="cuda"):
    """Hash tables (tab1, tab2) on the device for a named family
    ("multiply_add_shift", "multiply_shift", "tabulation")."""
    torch = _torch()
    kd = keys_tensor(keys, device)
    d = kd.shape[0]
    tab1 = torch.empty((d, n_rows), dtype=torch.int32, device=device)
    tab2 = torch.empty((d, n_cols), dtype=torch.int32, device=device)
    cmm_hash_family(HASH_FAMILIES[family], kd, d, n_rows, n_cols, log2b, tab1, tab2)
    return tab1, tab2


def keys_tensor(keys: np.ndarray, device="cuda"):
    """uint64[d][4][2] hash keys -> int64 device tensor with the same bits."""
    torch = _torch()
    k = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64)).view(np.int64)
    return torch.from_numpy(k.copy()).to(device)


def make_problem(A, B, d, log2b, *, keys=None, tab1=None, tab2=None, p=None, C_hat=None,
                 compute="f64", estimator="median") -> Problem:
    fn = "make_problem"
    torch = _torch()
    _like(A, fn, "A", _floats())
    _need(A.dim() == 2 and B.dim() == 2, fn, "A and B must be matrices")
    _like(B, fn, "B", (A.dtype,))
    _need(B.shape[0] == A.shape[1], fn,
          f"inner dimensions differ: A is {tuple(A.shape)}, B is {tuple(B.shape)}")
    n_rows, n_cols = A.shape[0], B.shape[1]
    if keys is not None:
        _like(keys, fn, "keys", (torch.int64,), min_numel=8 * d)
    _tables(fn, tab1, tab2, d, n_rows, n_cols)
    if p is not None:
        _sketch_p(fn, p, d, log2b)
    if C_hat is not None:
        _like(C_hat, fn, "C_hat", _floats(), (n_rows, n_cols))
    pr = Problem()
    pr.n_rows, pr.n_inner = A.shape
    pr.n_cols = B.shape[1]
    pr.A, pr.lda = _ptr(A, True), A.stride(0)
    pr.B, pr.ldb = _ptr(B, True), B.stride(0)
    pr.in_dtype = _dtype_code(A)
    pr.compute = _COMPUTE[compute]
    pr.d, pr.log2b = d, log2b
    pr.estimator = CMM_MEDIAN if estimator == "median" else CMM_MEAN
    pr.keys = _ptr(keys)
    pr.tab1, pr.tab2 = _ptr(tab1), _ptr(tab2)
    pr.p = _ptr(p)
    if C_hat is not None:
        pr.C_hat, pr.out_dtype, pr.ldc = _ptr(C_hat, True), _dtype_code(C_hat), C_hat.stride(0)
    # the struct holds raw device pointers: keep the tensors alive with it
    pr._tensors = (A, B, keys, tab1, tab2, p, C_hat)
    return pr


class Estimate:
    """Result of ``estimate``: C_hat, the sketch p and the hash tables."""

    def __init__(self, C_hat, p, tab1, tab2):
        self.C_hat, self.p, self.tab1, self.tab2 = C_hat, p, tab1, tab2


def estimate(A, B, d: int, log2b: int, *, keys=None, tab1=None, tab2=None,
             compute: str = "f64", estimator: str = "median", out_dtype=None,
             dense: bool = True, workspace=None, static_scratch: bool = False,
             stream=None) -> Estimate:
    """Compressed product of A (n_rows x n_inner) and B (n_inner x n_cols).

    Give either ``keys`` (uint64[d][4][2], numpy or an int64 device tensor)
    or explicit tables ``tab1`` / ``tab2`` (int32 device tensors).  With
    ``static_scratch`` the library's static scratch replaces the workspace
    (cmm_estimate_static)."""
    torch = _torch()
    dev = A.device
    n_rows, n_cols = A.shape[0], B.shape[1]
    if keys is not None and not hasattr(keys, "data_ptr"):
        keys = keys_tensor(keys, dev)
    if keys is not None:
        tab1 = torch.empty((d, n_rows), dtype=torch.int32, device=dev)
        tab2 = torch.empty((d, n_cols), dtype=torch.int32, device=dev)
    p = torch.empty((d, 1 << log2b), dtype=torch.float64, device=dev)
    C_hat = None
    if dense:
        C_hat = torch.empty((n_rows, n_cols), dtype=out_dtype or A.dtype, device=dev)
    pr = make_problem(A, B, d, log2b, keys=keys, tab1=tab1, tab2=tab2, p=p, C_hat=C_hat,
                      compute=compute, estimator=estimator)
    if static_scratch:
        cmm_estimate_static(pr, stream)
        return Estimate(C_hat, p, tab1, tab2)
    nbytes = cmm_workspace_size(pr)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    cmm_estimate(pr, workspace, nbytes, stream)
    return Estimate(C_hat, p, tab1, tab2)


class Batch:
    """A planned batch of problems (``cmm_batch``): all Compress work of the
    batch runs in one persistent launch.  Keeps the problems (and so their
    tensors) alive; ``run`` enqueues one estimate of every problem and can be
    captured into a graph."""

    def __init__(self, problems):
        self._problems = list(problems)
        arr = (Problem * len(self._problems))(*self._problems)
        h = ctypes.c_void_p()
        _check("cmm_batch_create", lib().cmm_batch_create(arr, len(self._problems), ctypes.byref(h)))
        self._h = h

    def workspace_size(self) -> int:
        n = ctypes.c_size_t(0)
        _check("cmm_batch_workspace_size", lib().cmm_batch_workspace_size(self._h, ctypes.byref(n)))
        return n.value

    def workspace(self, device="cuda"):
        """A fresh workspace tensor of the required size (256-byte aligned)."""
        torch = _torch()
        return torch.empty(max(self.workspace_size(), 1), dtype=torch.uint8, device=device)

    def autotune(self, workspace, stream=None) -> dict:
        _check("cmm_batch_autotune", lib().cmm_batch_autotune(
            self._h, _ptr(workspace), workspace.numel(), _stream(stream)))
        return self.config()

    def set_config(self, log2_blo: int, k_per_item: int, wg_per_cu: int, order: int,
                   radix: int = 16) -> None:
        _check("cmm_batch_set_config",
               lib().cmm_batch_set_config(self._h, log2_blo, k_per_item, wg_per_cu, order, radix))

    def config(self) -> dict:
        v = [ctypes.c_int(0) for _ in range(6)]
        _check("cmm_batch_get_config", lib().cmm_batch_get_config(self._h, *[ctypes.byref(x) for x in v]))
        return {"log2_blo": v[0].value, "k_per_item": v[1].value, "wg_per_cu": v[2].value,
                "order": ["largest first", "round robin"][v[3].value], "radix": v[4].value,
                "source": ["default", "tuned", "cache", "set"][v[5].value]}

    def run(self, workspace, stream=None) -> None:
        _check("cmm_estimate_batched", lib().cmm_estimate_batched(
            self._h, _ptr(workspace), workspace.numel(), _stream(stream)))

    def close(self) -> None:
        if self._h is not None and self._h.value:
            lib().cmm_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_batch(pairs, *, compute: str = "f32", estimator: str = "median", dense: bool = True):
    """Batch of (A, B, d, log2b, keys) tuples.  Returns (Batch, [Estimate])
    whose outputs are filled by every ``Batch.run``."""
    torch = _torch()
    problems, results = [], []
    for A, B, d, log2b, keys in pairs:
        dev = A.device
        if not hasattr(keys, "data_ptr"):
            keys = keys_tensor(keys, dev)
        tab1 = torch.empty((d, A.shape[0]), dtype=torch.int32, device=dev)
        tab2 = torch.empty((d, B.shape[1]), dtype=torch.int32, device=dev)
        p = torch.empty((d, 1 << log2b), dtype=torch.float64, device=dev)
        C_hat = torch.empty((A.shape[0], B.shape[1]), dtype=A.dtype, device=dev) if dense else None
        problems.append(make_problem(A, B, d, log2b, keys=keys, tab1=tab1, tab2=tab2, p=p,
                                     C_hat=C_hat, compute=compute, estimator=estimator))
        results.append(Estimate(C_hat, p, tab1, tab2))
    return Batch(problems), results


def tables_to_numpy(tab) -> np.ndarray:
    """int32 device table -> uint32 numpy array with the same bits."""
    return tab.cpu().numpy().view(np.uint32)


def effective_rate(n_rows: int, n_inner: int, n_cols: int, seconds: float) -> float:
    """2 n_rows n_inner n_cols / seconds (DGEMM-equivalent flop rate)."""
    return 2.0 * n_rows * n_inner * n_cols / seconds if seconds > 0 else math.inf
