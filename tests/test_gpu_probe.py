"""The gather probe (a measurement aid beside the extract) on the GPU: every
index it draws lies inside the table, whatever its length, and the sink is
written only in the one case the kernel reserves for it."""
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
