"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every function the header declares, and argument checks return
CMM_EINVAL before anything touches the device."""
import ctypes
import os
import re

import pytest

import paper_2601_09477_amd as cmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "cmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cmm_[a-z_]+)\s*\(", src)))


def _lib_or_skip():
    if not os.path.exists(cmm.LIB_PATH):
        pytest.skip("libcmm.so not built")
    return cmm.lib()


def test_header_declares_the_boundary():
    fns = _header_functions()
    for name in ["cmm_hash", "cmm_sketch", "cmm_fwht", "cmm_accumulate", "cmm_extract",
                 "cmm_estimate", "cmm_workspace_size"]:
        assert name in fns
    assert set(fns) == set(cmm.EXPORTED)


def test_library_exports_every_header_symbol():
    L = _lib_or_skip()
    for name in _header_functions():
        assert hasattr(L, name), name
    assert L.cmm_abi_version() == 2
    assert L.cmm_status_string(1) == b"CMM_EINVAL"


def test_problem_struct_layout_matches_header():
    # offsets of the C struct on x86-64 (int64 / pointer = 8, enum / int = 4)
    P = cmm.Problem
    assert P.A.offset == 24 and P.lda.offset == 32 and P.B.offset == 40
    assert P.in_dtype.offset == 56 and P.estimator.offset == 72 and P.keys.offset == 80
    assert P.C_hat.offset == 112 and P.out_dtype.offset == 120 and P.ldc.offset == 128
    assert ctypes.sizeof(P) == 136


@pytest.mark.parametrize("call", [
    lambda L: L.cmm_hash(None, 0, 4, 4, 8, None, None, None),          # d = 0
    lambda L: L.cmm_hash(None, 3, 4, 4, 31, None, None, None),         # log2b too large
    lambda L: L.cmm_hash(None, 3, 4, 4, 8, None, None, None),          # null keys
    lambda L: L.cmm_hash(1, 3, 1 << 33, 4, 8, 1, 1, None),              # beyond hash domain
    lambda L: L.cmm_hash_family(3, 1, 3, 4, 4, 8, 1, 1, None),          # unknown family
    lambda L: L.cmm_hash_family(-1, 1, 3, 4, 4, 8, 1, 1, None),         # unknown family
    lambda L: L.cmm_hash_family(2, None, 3, 4, 4, 8, 1, 1, None),       # null keys
    lambda L: L.cmm_hash_family(1, 1, 0, 4, 4, 8, 1, 1, None),          # d = 0
    lambda L: L.cmm_hash_family(2, 1, 3, 4, 4, 8, 1, None, None),       # null tab2
    lambda L: L.cmm_sketch(2, 1, 0, 4, 4, 4, 1, 1, 8, 0, 1, 1, 0, None),   # bad side
    lambda L: L.cmm_sketch(0, 1, 2, 4, 4, 4, 1, 1, 8, 0, 1, 1, 0, None),   # bf16 not a sketch type
    lambda L: L.cmm_sketch(0, 1, 0, 4, 4, 4, 1, 1, 8, 0, 1, 1, 3, None),   # fp16 not an output type
    lambda L: L.cmm_sketch(0, 1, 0, 4, 4, 3, 1, 1, 8, 0, 1, 1, 0, None),   # ld < cols
    lambda L: L.cmm_sketch(0, 1, 0, 4, 4, 4, 1, 1, 8, 3, 2, 1, 0, None),   # k0 + kc > inner
    lambda L: L.cmm_fwht(1, 0, 4, 8, 3.0, None),                        # scale not a power of 2
    lambda L: L.cmm_fwht(1, 0, 4, 0, 1.0, None),                        # log2b = 0
    lambda L: L.cmm_fwht(None, 0, 4, 8, 1.0, None),                     # null x
    lambda L: L.cmm_accumulate(None, 1, 0, 3, 2, 8, 1, None),           # null X
    lambda L: L.cmm_extract(1, 1, 1, 4, 8, 8, 8, 0, 1, 0, 8, None),     # median with even d
    lambda L: L.cmm_extract(1, 1, 1, 3, 8, 8, 8, 0, 1, 0, 7, None),     # ldc < n_cols
    lambda L: L.cmm_gather_probe(None, 10, 10, 0, 1, None, None),      # null table
    lambda L: L.cmm_gather_probe(1, 10, 10, 0, None, None, None),      # null sink
    lambda L: L.cmm_gather_probe(1, 0, 10, 0, 1, None, None),          # empty table
    lambda L: L.cmm_gather_probe(1, (1 << 32) + 1, 10, 0, 1, None, None),  # table too long
    lambda L: L.cmm_gather_probe(1, 10, 0, 0, 1, None, None),          # no gathers
    lambda L: L.cmm_gather_probe(1, 10, (1 << 40) + 1, 0, 1, None, None),  # too many
    lambda L: L.cmm_extract(1, 1, 1, 3, 8, 8, 8, 5, 1, 0, 8, None),     # unknown estimator
    lambda L: L.cmm_extract_entries(1, 1, 1, 4, 8, 8, 8, 0, 1, 1, 4, 1, 0, None),  # median, even d
    lambda L: L.cmm_extract_entries(1, 1, 1, 3, 8, 8, 8, 0, None, 1, 4, 1, 0, None),  # rows null
    lambda L: L.cmm_extract_entries(1, 1, 1, 3, 8, 8, 8, 0, 1, 1, -1, 1, 0, None),  # count < 0
    lambda L: L.cmm_extract_heavy(1, 1, 1, 3, 8, 8, 8, 0, float("nan"), 1, 1, 1, 0, 4, 1, None),
    lambda L: L.cmm_extract_heavy(1, 1, 1, 3, 8, 8, 8, 0, 1.0, 1, 1, 1, 0, 4, None, None),  # count
    lambda L: L.cmm_extract_heavy(1, 1, 1, 3, 8, 8, 8, 0, 1.0, None, 1, 1, 0, 4, 1, None),  # list
    lambda L: L.cmm_extract_heavy(1, 1, 1, 3, 8, 8, 8, 0, 1.0, 1, 1, 1, 2, 4, 1, None),  # bf16 out
    lambda L: L.cmm_extract_reps(1, 1, 1, 0, 8, 8, 8, 1, 1, 4, 1, 0, None),       # d = 0
    lambda L: L.cmm_extract_reps(1, 1, 1, 4, 8, 8, 8, None, 1, 4, 1, 0, None),    # rows null
    lambda L: L.cmm_extract_reps(1, 1, 1, 4, 8, 8, 8, 1, 1, -2, 1, 0, None),      # count < 0
    lambda L: L.cmm_extract_reps(1, 1, 1, 4, 8, 8, 8, 1, 1, 4, 1, 3, None),       # f16 out
    lambda L: L.cmm_correctness_counts(1, 2, 8, 1, 8, 8, 8, 1, 1, 1, 0.5, 0.1, 1, None),  # bf16
    lambda L: L.cmm_correctness_counts(1, 0, 7, 1, 8, 8, 8, 1, 1, 1, 0.5, 0.1, 1, None),  # ldh
    lambda L: L.cmm_correctness_counts(1, 0, 8, 1, 8, 8, 8, 1, 1, 1, -1.0, 0.1, 1, None),  # thr
    lambda L: L.cmm_correctness_counts(1, 0, 8, 1, 8, 8, 8, 1, 1, 1, 0.5, float("nan"), 1,
                                       None),                                       # tol NaN
    lambda L: L.cmm_correctness_counts(1, 0, 8, 1, 8, 8, 8, 1, 1, 1, 0.5, 0.1, None, None),  # counts
    lambda L: L.cmm_correctness_counts(1, 0, 8, 1, 8, 8, 8, None, 1, 1, 0.5, 0.1, 1, None),  # big
    lambda L: L.cmm_fft(1, 2, 4, 0, 0, 1.0, None),                      # log2n = 0
    lambda L: L.cmm_fft(1, 2, 4, 25, 0, 1.0, None),                     # log2n > 24
    lambda L: L.cmm_fft(1, 2, 4, 8, 2, 1.0, None),                      # inverse not 0 / 1
    lambda L: L.cmm_fft(1, 2, 4, 8, 0, float("inf"), None),             # scale not finite
    lambda L: L.cmm_fft(1, 1, 4, 13, 0, 1.0, None),                     # in place above 2^12
    lambda L: L.cmm_fft(None, 2, 4, 8, 0, 1.0, None),                   # null
    lambda L: L.cmm_extract_cyclic(1, 1, 1, 4, 8, 8, 8, 0, 1, 0, 8, None),   # median, even d
    lambda L: L.cmm_extract_cyclic(1, 1, 1, 3, 8, 8, 8, 0, 1, 0, 7, None),   # ldc < n_cols
    lambda L: L.cmm_extract_cyclic(1, 1, 1, 3, 8, 8, 8, 0, None, 0, 8, None),  # C_hat null
])
def test_invalid_arguments_rejected_on_host(call):
    L = _lib_or_skip()
    assert call(L) == cmm.CMM_EINVAL
    assert len(L.cmm_last_error()) > 0


def _problem(**kw):
    pr = cmm.Problem()
    pr.n_rows, pr.n_inner, pr.n_cols = 8, 8, 8
    pr.A, pr.lda, pr.B, pr.ldb = 1, 8, 1, 8
    pr.in_dtype, pr.compute, pr.d, pr.log2b = cmm.CMM_F64, cmm.CMM_F64, 3, 10
    pr.estimator, pr.tab1, pr.tab2 = cmm.CMM_MEDIAN, 1, 1
    for k, v in kw.items():
        setattr(pr, k, v)
    return pr


@pytest.mark.parametrize("kw", [
    dict(d=4), dict(log2b=0), dict(lda=7), dict(in_dtype=cmm.CMM_F32),
    dict(compute=9), dict(A=None), dict(tab1=None), dict(C_hat=1, ldc=7),
    dict(n_rows=(1 << 32) + 1),
])
def test_problem_validation(kw):
    L = _lib_or_skip()
    n = ctypes.c_size_t(0)
    assert L.cmm_workspace_size(ctypes.byref(_problem(**kw)), ctypes.byref(n)) == cmm.CMM_EINVAL
    assert L.cmm_estimate(ctypes.byref(_problem(**kw)), None, 0, None) == cmm.CMM_EINVAL


@pytest.mark.parametrize("kw", [
    dict(compute=cmm.CMM_BF16, log2b=13),                                   # b_lo = 2^14 needs b >= 2^14
    dict(compute=cmm.CMM_F16, log2b=16, n_rows=16384, lda=8),               # zero-pad offset in 15 bits
    dict(compute=cmm.CMM_BF16, log2b=16, n_cols=16384, ldb=16384),
])
def test_precision_form_limits(kw):
    L = _lib_or_skip()
    n = ctypes.c_size_t(0)
    assert L.cmm_workspace_size(ctypes.byref(_problem(**kw)), ctypes.byref(n)) == cmm.CMM_EUNSUPPORTED
    assert b"precision form" in L.cmm_last_error()


@pytest.mark.parametrize("kw,status", [
    (dict(compute=cmm.CMM_F32), cmm.CMM_EUNSUPPORTED),            # the FFT form is float64 only
    (dict(in_dtype=cmm.CMM_F32, compute=cmm.CMM_F32), cmm.CMM_EUNSUPPORTED),
    (dict(d=4), cmm.CMM_EINVAL),
    (dict(tab1=None), cmm.CMM_EINVAL),
])
def test_fft_form_validation(kw, status):
    L = _lib_or_skip()
    n = ctypes.c_size_t(0)
    pr = _problem(**kw)
    assert L.cmm_fft_workspace_size(ctypes.byref(pr), ctypes.byref(n)) == status
    assert L.cmm_estimate_fft(ctypes.byref(pr), 1, 1 << 40, None) == status


def test_fft_form_short_workspace():
    L = _lib_or_skip()
    pr = _problem(n_rows=64, n_inner=32, n_cols=48, lda=32, ldb=48)
    n = ctypes.c_size_t(0)
    assert L.cmm_fft_workspace_size(ctypes.byref(pr), ctypes.byref(n)) == cmm.CMM_OK
    assert L.cmm_estimate_fft(ctypes.byref(pr), 1, n.value - 1, None) == cmm.CMM_ENOMEM


@pytest.mark.parametrize("kw,status", [
    (dict(estimator=cmm.CMM_MEDIAN), cmm.CMM_EUNSUPPORTED),       # the adjoint is of the mean
    (dict(compute=cmm.CMM_BF16, log2b=14), cmm.CMM_EUNSUPPORTED),
    (dict(log2b=10), cmm.CMM_EUNSUPPORTED),                      # b_lo >= 2^11
    (dict(d=0), cmm.CMM_EINVAL),
    (dict(A=None), cmm.CMM_EINVAL),
])
def test_backward_validation(kw, status):
    L = _lib_or_skip()
    base = dict(estimator=cmm.CMM_MEAN, log2b=12)
    base.update(kw)
    n = ctypes.c_size_t(0)
    pr = _problem(**base)
    assert L.cmm_backward_workspace_size(ctypes.byref(pr), ctypes.byref(n)) == status
    assert L.cmm_estimate_backward(ctypes.byref(pr), 1, 8, 1, 8, 1, 8, 1, 1 << 40, None) == status


@pytest.mark.parametrize("args", [
    (None, 8, 1, 8, 1, 8),   # W null
    (1, 7, 1, 8, 1, 8),      # ldw < n_cols
    (1, 8, 1, 7, 1, 8),      # ldda < n_inner
    (1, 8, 1, 8, 1, 7),      # lddb < n_cols
    (1, 8, None, 8, 1, 8),   # dA null
])
def test_backward_arguments_rejected_on_host(args):
    L = _lib_or_skip()
    pr = _problem(estimator=cmm.CMM_MEAN, log2b=12)
    assert L.cmm_estimate_backward(ctypes.byref(pr), *args, 1, 1 << 40, None) == cmm.CMM_EINVAL


def test_backward_short_workspace():
    L = _lib_or_skip()
    pr = _problem(estimator=cmm.CMM_MEAN, log2b=12, n_rows=64, n_inner=32, n_cols=48, lda=32,
                  ldb=48)
    n = ctypes.c_size_t(0)
    assert L.cmm_backward_workspace_size(ctypes.byref(pr), ctypes.byref(n)) == cmm.CMM_OK
    assert L.cmm_estimate_backward(ctypes.byref(pr), 1, 48, 1, 32, 1, 48, 1, n.value - 1,
                                   None) == cmm.CMM_ENOMEM


def test_workspace_size_and_short_workspace():
    L = _lib_or_skip()
    n = ctypes.c_size_t(0)
    pr = _problem(n_rows=256, n_inner=256, n_cols=256, lda=256, ldb=256, log2b=12, d=5)
    assert L.cmm_workspace_size(ctypes.byref(pr), ctypes.byref(n)) == cmm.CMM_OK
    assert n.value > 5 * 4096 * 8
    # a workspace one byte short is refused before any launch
    assert L.cmm_estimate(ctypes.byref(pr), 1, n.value - 1, None) == cmm.CMM_ENOMEM


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(cmm, "_lib", None)
    monkeypatch.setattr(cmm, "LIB_PATH", "/nonexistent/libcmm.so")
    with pytest.raises(cmm.CmmError):
        cmm.lib()


def _profiled_names():
    """Names the library's timing scopes are constructed with, from its sources."""
    csrc = os.path.join(ROOT, "paper_2601_09477_amd", "csrc")
    names = set()
    for f in os.listdir(csrc):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(csrc, f)) as fh:
                names |= set(re.findall(r'ProfScope\s+\w+\("(\w+)"', fh.read()))
    return names


def test_profile_names_listed_in_header():
    with open(os.path.join(ROOT, "include", "cmm.h")) as fh:
        hdr = fh.read()
    block = hdr[hdr.index("Tracing for measurement"):hdr.index("void cmm_profile_enable")]
    listed = set(re.findall(r'"(\w+)"', block))
    assert _profiled_names() == listed


def test_profile_only_validates_names():
    L = _lib_or_skip()
    L.cmm_last_error.restype = ctypes.c_char_p
    assert L.cmm_profile_only(b"no_such_kernel") == 1          # CMM_EINVAL
    assert b"no_such_kernel" in L.cmm_last_error()
    for name in sorted(_profiled_names()):
        assert L.cmm_profile_only(name.encode()) == 0, name
    assert L.cmm_profile_only(None) == 0


def test_gather_probe_binding_rejects_strided_tables():
    import torch
    t = torch.zeros((4, 4), dtype=torch.float64).t()
    with pytest.raises(ValueError):
        cmm.cmm_gather_probe(t, 16, torch.zeros(1, dtype=torch.float64))
    with pytest.raises(TypeError):
        cmm.cmm_gather_probe(torch.zeros(4, dtype=torch.float32), 16,
                             torch.zeros(1, dtype=torch.float64))


@pytest.mark.parametrize("kw", [
    dict(log2b=25),                 # the transform's two LDS-tile passes stop at 2^24 points
    dict(log2b=30, d=1),
])
def test_fft_form_transform_length_limit(kw):
    # refused before any launch (a pass longer than the tile used to divide
    # by zero on the host)
    L = _lib_or_skip()
    n = ctypes.c_size_t(0)
    pr = _problem(**kw)
    assert L.cmm_fft_workspace_size(ctypes.byref(pr), ctypes.byref(n)) == cmm.CMM_EUNSUPPORTED
    assert b"log2b <= 24" in L.cmm_last_error()
    assert L.cmm_estimate_fft(ctypes.byref(pr), 1, 1 << 40, None) == cmm.CMM_EUNSUPPORTED


# Buffers of 2^31 or more elements are refused on the host: the kernels'
# index arithmetic is not audited past that.  46341^2 > 2^31 > 46340^2.
@pytest.mark.parametrize("kw", [
    dict(n_rows=46341, n_inner=46341, n_cols=8, lda=46341, ldb=8),   # A
    dict(n_rows=8, n_inner=46341, n_cols=46341, lda=46341, ldb=46341),  # B
    dict(n_rows=46341, n_inner=8, n_cols=46341, lda=8, ldb=46341, C_hat=1,
         out_dtype=cmm.CMM_F64, ldc=46341),                          # C_hat
    dict(n_rows=8, n_inner=8, n_cols=8, lda=8, ldb=1 << 31),         # B's leading dimension
    dict(d=3, log2b=30),                                             # p: 3 x 2^30
    dict(d=9999, n_rows=1 << 18, n_inner=1, lda=1),                  # table d x n_rows
])
def test_problem_beyond_index_range(kw):
    L = _lib_or_skip()
    n = ctypes.c_size_t(0)
    pr = _problem(**kw)
    assert L.cmm_workspace_size(ctypes.byref(pr), ctypes.byref(n)) == cmm.CMM_EUNSUPPORTED
    assert b"2^31" in L.cmm_last_error()
    assert L.cmm_estimate(ctypes.byref(pr), 1, 1 << 62, None) == cmm.CMM_EUNSUPPORTED
    assert L.cmm_estimate_fft(ctypes.byref(pr), 1, 1 << 62, None) == cmm.CMM_EUNSUPPORTED


def test_problem_just_inside_index_range():
    # 46340^2 < 2^31: the size checks pass (only the workspace is sized)
    L = _lib_or_skip()
    n = ctypes.c_size_t(0)
    pr = _problem(n_rows=46340, n_inner=46340, n_cols=8, lda=46340, ldb=8)
    assert L.cmm_workspace_size(ctypes.byref(pr), ctypes.byref(n)) == cmm.CMM_OK


@pytest.mark.parametrize("call", [
    lambda L: L.cmm_sketch(0, 1, 0, 46341, 46341, 46341, 1, 1, 8, 0, 1, 1, 0, None),  # M
    lambda L: L.cmm_sketch(0, 1, 0, 8, 1 << 20, 1 << 20, 1, 9, 20, 0, 1 << 20, 1, 0, None),  # out
    lambda L: L.cmm_fwht(1, 0, 1 << 12, 20, 1.0, None),                  # 2^32 elements
    lambda L: L.cmm_accumulate(1, 1, 0, 9, 1 << 12, 20, 1, None),
    lambda L: L.cmm_extract(1, 1, 1, 3, 46341, 46341, 8, 0, 1, 0, 46341, None),
    lambda L: L.cmm_extract_cyclic(1, 1, 1, 3, 46341, 46341, 8, 0, 1, 0, 46341, None),
    lambda L: L.cmm_extract_reps(1, 1, 1, 1000, 8, 8, 8, 1, 1, 1 << 22, 1, 0, None),
    lambda L: L.cmm_extract_entries(1, 1, 1, 3, 8, 8, 30, 0, 1, 1, 4, 1, 0, None),  # p 3 x 2^30
    lambda L: L.cmm_correctness_counts(1, 0, 46341, 1, 46341, 46341, 46341, 1, 1, 1, 0.5, 0.1,
                                       1, None),
    lambda L: L.cmm_fft(1, 2, 1 << 12, 20, 0, 1.0, None),
])
def test_standalone_calls_beyond_index_range(call):
    L = _lib_or_skip()
    assert call(L) == cmm.CMM_EUNSUPPORTED
    assert b"2^31" in L.cmm_last_error()


def test_backward_beyond_index_range():
    L = _lib_or_skip()
    pr = _problem(estimator=cmm.CMM_MEAN, log2b=12)
    # W with a leading dimension of 2^28 over 8 rows: 2^31 elements
    assert L.cmm_estimate_backward(ctypes.byref(pr), 1, 1 << 28, 1, 8, 1, 8, 1, 1 << 40,
                                   None) == cmm.CMM_EUNSUPPORTED
