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
