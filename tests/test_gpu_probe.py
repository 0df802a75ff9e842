"""The measurement aids on the GPU.  The gather probe: every index it draws
lies inside the table, whatever its length, and the sink is written only in
the one case the kernel reserves for it.  The timing filter: it brackets
exactly the named kernel's launches."""
import pytest

import paper_2601_09477_amd as cmm
from tests.gpu_util import announce, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch().cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()


@pytest.mark.parametrize("length,gathers", [(1, 1), (1000, 10000), (9 << 16, 1 << 20),
                                            ((1 << 20) + 3, 3 * 16384 + 1)])
def test_gather_probe_in_bounds(length, gathers):
    announce(f"gather probe len={length} gathers={gathers}")
    T = torch()
    # one guard value on each side of the table: the probe must read none
    buf = T.full((length + 2,), float("nan"), dtype=T.float64, device="cuda")
    table = buf[1:length + 1]
    table.fill_(1.0)
    sink = T.zeros(1, dtype=T.float64, device="cuda")
    issued = cmm.cmm_gather_probe(table, gathers, sink, seed=7)
    T.cuda.synchronize()
    assert issued >= gathers and issued % 16384 == 0
    # every gathered value is 1.0, so no per-thread sum is the sink's value
    assert sink.item() == 0.0


def test_profile_only_brackets_one_kernel():
    """cmm_profile_only: while it names a kernel, only that kernel's launches
    are timed; NULL times every kernel again."""
    from workloads import draw_keys
    announce("profile_only over one estimate")
    T = torch()
    n, d, log2b = 256, 3, 12
    g = T.Generator().manual_seed(5)
    A = T.randint(-1, 2, (n, n), generator=g).to(T.float64).cuda()
    B = T.randint(-1, 2, (n, n), generator=g).to(T.float64).cuda()
    keys = draw_keys(d, 3)
    try:
        cmm.cmm_profile_only("compress")
        cmm.cmm_profile_enable(True)
        cmm.estimate(A, B, d, log2b, keys=keys, compute="f64")
        T.cuda.synchronize()
        ms, launches = cmm.cmm_profile_query("compress")
        assert launches == 1 and ms > 0.0
        assert cmm.cmm_profile_query("extract") == (0.0, 0)
        assert cmm.cmm_profile_query("hash") == (0.0, 0)
        cmm.cmm_profile_only(None)
        cmm.cmm_profile_enable(True)
        cmm.estimate(A, B, d, log2b, keys=keys, compute="f64")
        T.cuda.synchronize()
        assert cmm.cmm_profile_query("compress")[1] == 1
        assert cmm.cmm_profile_query("extract")[1] == 1
        assert cmm.cmm_profile_query("hash")[1] == 1
    finally:
        cmm.cmm_profile_only(None)
        cmm.cmm_profile_enable(False)
