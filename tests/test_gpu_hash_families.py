"""Alternative hash families on the GPU (multiply-shift, simple tabulation):
tables bit-exact against the oracle, and the full estimate with tables of
each family against the oracle's plain definition."""
import numpy as np
import pytest

import oracle as O
import paper_2601_09477_amd as cmm
from workloads import draw_family_keys, small_random
from tests.gpu_util import announce, dev, host, torch

pytestmark = pytest.mark.gpu

FAMILIES = ["multiply_add_shift", "multiply_shift", "tabulation"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch().cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("d,n_rows,n_cols,log2b", [
    (1, 1, 1, 1), (3, 257, 70001, 13), (5, 66000, 300, 20), (2, 1000, 999, 30)])
def test_family_tables_bit_exact(family, d, n_rows, n_cols, log2b):
    # 70001 and 66000 indices reach the third byte of the key
    announce(f"hash family {family} d={d} n={n_rows}x{n_cols} log2b={log2b}")
    keys = draw_family_keys(family, d, 17 * d + log2b)
    tab1, tab2 = cmm.family_tables(family, keys, n_rows, n_cols, log2b)
    r1, r2 = O.hash_tables_family(family, keys, n_rows, n_cols, log2b)
    assert np.array_equal(cmm.tables_to_numpy(tab1), r1)
    assert np.array_equal(cmm.tables_to_numpy(tab2), r2)


@pytest.mark.parametrize("family", FAMILIES[1:])
def test_estimate_with_family_tables(family):
    # integer inputs: the float64 path is exact
    announce(f"estimate with {family} tables")
    T = torch()
    nr, ni, nc, log2b, d = 300, 140, 260, 14, 5
    w = small_random(nr, ni, nc, log2b, d, seed=4, integer=True)
    keys = draw_family_keys(family, d, 303)
    t1, t2 = O.hash_tables_family(family, keys, nr, nc, log2b)
    p_ref = O.bucket_sums(O.product(w.A, w.B), t1, t2, log2b)
    C_ref = O.extract(p_ref, t1, t2, "median")
    tab1, tab2 = cmm.family_tables(family, keys, nr, nc, log2b)
    res = cmm.estimate(dev(w.A), dev(w.B), d, log2b, tab1=tab1, tab2=tab2)
    assert np.array_equal(cmm.tables_to_numpy(res.tab1), t1)
    assert np.array_equal(host(res.p), p_ref)
    assert np.array_equal(host(res.C_hat), C_ref)
