"""cmm_estimate_static, the entry point that allocates nothing (GPU): its
scratch is the library's static device array instead of a caller's
workspace.  Two calls in a row, the second on a smaller problem (the array
still holds the first call's contents), each against cmm_estimate with a
fresh workspace on the same inputs, bit for bit (same kernels, same
fixed-order reductions); a problem whose scratch exceeds the array is
refused before any launch."""
import numpy as np
import pytest

import oracle as O
import paper_2601_09477_amd as cmm
from workloads import draw_keys, small_random
from tests.gpu_util import announce, dev, host, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch().cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()


def _both(w, compute="f64"):
    T = torch()
    dt = T.float64 if compute == "f64" else T.float32
    A, B = dev(w.A, dt), dev(w.B, dt)
    ref = cmm.estimate(A, B, w.d, w.log2b, keys=w.keys, compute=compute)
    got = cmm.estimate(A, B, w.d, w.log2b, keys=w.keys, compute=compute, static_scratch=True)
    T.cuda.synchronize()
    return ref, got


@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_static_scratch_matches_workspace(compute):
    big = small_random(1000, 700, 900, 14, 7, seed=41)
    small = small_random(120, 90, 70, 12, 5, seed=42)
    for w in (big, small):
        announce(f"estimate static scratch {compute} {w.name}")
        ref, got = _both(w, compute)
        assert np.array_equal(host(got.p), host(ref.p))
        assert np.array_equal(host(got.C_hat), host(ref.C_hat))
        assert np.array_equal(cmm.tables_to_numpy(got.tab1), cmm.tables_to_numpy(ref.tab1))
    # the small problem against the oracle as well (float64: within 1e-9 ||C||_F / n)
    if compute == "f64":
        t1, t2 = O.hash_tables(small.keys, 120, 70, small.log2b)
        C = O.product(small.A, small.B)
        p_ref = O.bucket_sums(C, t1, t2, small.log2b)
        assert np.abs(host(got.p) - p_ref).max() <= 1e-9 * np.linalg.norm(C) / 90


def test_static_scratch_rejects_large_problems():
    announce("estimate static scratch: too large")
    T = torch()
    n, d, log2b = 2048, 9, 16
    A = T.zeros((n, n), dtype=T.float64, device="cuda")
    with pytest.raises(cmm.CmmError) as e:
        cmm.estimate(A, A, d, log2b, keys=draw_keys(d, 1), static_scratch=True)
    assert e.value.status == cmm.CMM_EUNSUPPORTED
