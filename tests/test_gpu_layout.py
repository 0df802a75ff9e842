"""The binding refuses tensor layouts the library cannot address (GPU): a
buffer must be contiguous, and a matrix given with a leading dimension needs
unit stride along its rows.  An expanded view covers less memory than the
sizes describe, so passing it on would send the kernels past its end; the
error is raised before any launch."""
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


def test_layouts_rejected_before_launch():
    announce("binding layout checks")
    T = torch()
    d, n, log2b = 3, 64, 10
    keys = cmm.keys_tensor(draw_keys(d, 1), "cuda")
    tab_row = T.zeros((1, n), dtype=T.int32, device="cuda")
    expanded = tab_row.expand(d, n)                       # stride 0 over d
    good = T.empty((d, n), dtype=T.int32, device="cuda")
    with pytest.raises(cmm.CmmError):
        cmm.cmm_hash(keys, d, n, n, log2b, expanded, good)
    A = T.randn(n, n, dtype=T.float64, device="cuda")
    with pytest.raises(cmm.CmmError):
        cmm.estimate(A.t(), A, d, log2b, keys=draw_keys(d, 1))       # column-major
    with pytest.raises(cmm.CmmError):
        cmm.estimate(T.randn(n, 2 * n, dtype=T.float64, device="cuda")[:, ::2], A, d, log2b,
                     keys=draw_keys(d, 1))                            # stride 2 along rows
    # a row-major view with a larger leading dimension is fine
    wide = T.randn(n, 2 * n, dtype=T.float64, device="cuda")
    res = cmm.estimate(wide[:, :n], A, d, log2b, keys=draw_keys(d, 1))
    ref = cmm.estimate(wide[:, :n].contiguous(), A, d, log2b, keys=draw_keys(d, 1))
    T.cuda.synchronize()
    assert np.array_equal(res.C_hat.cpu().numpy(), ref.C_hat.cpu().numpy())


def test_shapes_and_dtypes_rejected_before_launch():
    # every tensor the library would read or write through is checked
    # against the problem's sizes and the input dtype before any launch
    announce("binding shape and dtype checks")
    T = torch()
    d, n, log2b = 3, 64, 10
    f64, f32, i32 = T.float64, T.float32, T.int32
    A = T.randn(n, 40, dtype=f64, device="cuda")
    B = T.randn(40, 48, dtype=f64, device="cuda")
    keys = draw_keys(d, 2)
    bad = [
        lambda: cmm.estimate(A, T.randn(39, 48, dtype=f64, device="cuda"), d, log2b, keys=keys),
        lambda: cmm.estimate(A, B.to(f32), d, log2b, keys=keys),
        lambda: cmm.estimate(A, B, d, log2b, tab1=T.zeros((d, n - 1), dtype=i32, device="cuda"),
                             tab2=T.zeros((d, 48), dtype=i32, device="cuda")),
        lambda: cmm.estimate(A, B, d, log2b, tab1=T.zeros((d, n), dtype=T.int64, device="cuda"),
                             tab2=T.zeros((d, 48), dtype=i32, device="cuda")),
    ]
    res = cmm.estimate(A, B, d, log2b, keys=keys)
    p, t1, t2 = res.p, res.tab1, res.tab2
    bad += [
        lambda: cmm.cmm_extract(p, t1, t2, d, n, 48, log2b, cmm.CMM_MEDIAN,
                                T.empty((n, 47), dtype=f64, device="cuda")),
        lambda: cmm.cmm_extract(p[:, :-1].contiguous(), t1, t2, d, n, 48, log2b, cmm.CMM_MEDIAN,
                                T.empty((n, 48), dtype=f64, device="cuda")),
        lambda: cmm.cmm_extract(p, t1, t2, d, n, 48, log2b, cmm.CMM_MEDIAN,
                                T.empty((n, 48), dtype=T.int32, device="cuda")),
    ]
    for q, call in enumerate(bad):
        with pytest.raises(cmm.CmmError):
            call()
        T.cuda.synchronize()


def test_row_major_views_with_a_leading_dimension():
    # Decompress into a view with a larger leading dimension writes the same
    # values as into a contiguous output, and leaves the columns past the
    # view untouched; a count sketch of such a view of A equals that of A
    announce("binding leading-dimension views")
    T = torch()
    d, n, log2b = 3, 64, 10
    A = T.randn(n, 40, dtype=T.float64, device="cuda")
    B = T.randn(40, 48, dtype=T.float64, device="cuda")
    res = cmm.estimate(A, B, d, log2b, keys=draw_keys(d, 3))
    wide = T.full((n, 80), 7.0, dtype=T.float64, device="cuda")
    cmm.cmm_extract(res.p, res.tab1, res.tab2, d, n, 48, log2b, cmm.CMM_MEDIAN, wide[:, :48])
    T.cuda.synchronize()
    assert np.array_equal(wide[:, :48].cpu().numpy(), res.C_hat.cpu().numpy())
    assert bool((wide[:, 48:] == 7.0).all())
    big = T.zeros((n, 72), dtype=T.float64, device="cuda")
    big[:, :40] = A
    kc = 8
    out_v = T.empty((d, kc, 1 << log2b), dtype=T.float64, device="cuda")
    out_c = T.empty_like(out_v)
    cmm.cmm_sketch(0, big[:, :40], n, 40, tab=res.tab1, d=d, log2b=log2b, k0=5, kc=kc, out=out_v)
    cmm.cmm_sketch(0, A, n, 40, tab=res.tab1, d=d, log2b=log2b, k0=5, kc=kc, out=out_c)
    T.cuda.synchronize()
    assert T.equal(out_v, out_c)
