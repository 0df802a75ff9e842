"""Precision form (bf16 / fp16 operands on MFMA, float32 accumulation,
float64 cross-k sum and inverse) against the float64 oracle (GPU).

Where every rounded quantity is an integer the low precision represents
exactly, the precision form is exact; otherwise the error is measured and
bounded (see the derivation in each test)."""
import numpy as np
import pytest

import oracle as O
import paper_2601_09477_amd as cmm
from workloads import draw_keys, planted_8192, small_random
from tests.gpu_util import announce, dev, host, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch().cuda.is_available():
        pytest.skip("no GPU")
    cmm.lib()


def _ref(w, n_rows, n_cols):
    t1, t2 = O.hash_tables(w.keys, n_rows, n_cols, w.log2b)
    C = O.product(w.A, w.B)
    return C, O.bucket_sums(C, t1, t2, w.log2b), t1, t2


@pytest.mark.parametrize("compute", ["f16", "bf16"])
def test_mfma_small_integers_exact(compute):
    # Entries in {-1, 0, 1} with 200 inner rows: every sketch value and
    # every transform intermediate is an integer of magnitude <= 200 * 16 <
    # 2^12 before the final float32 passes ... bf16 keeps 8 significant bits,
    # so it is exact only while |values| <= 256: use 32 inner rows for bf16.
    n_inner = 200 if compute == "f16" else 32
    announce(f"mfma {compute} small integers n_inner={n_inner}")
    rng = np.random.default_rng(21)
    A = rng.integers(-1, 2, size=(300, n_inner)).astype(np.float64)
    B = rng.integers(-1, 2, size=(n_inner, 260)).astype(np.float64)
    keys = draw_keys(3, 77)
    from types import SimpleNamespace
    w = SimpleNamespace(A=A, B=B, keys=keys, log2b=14, d=3)
    res = cmm.estimate(dev(A), dev(B), 3, 14, keys=keys, compute=compute)
    C, p_ref, t1, t2 = _ref(w, 300, 260)
    assert np.array_equal(host(res.p), p_ref)
    assert np.array_equal(host(res.C_hat), O.extract(p_ref, t1, t2, "median"))


@pytest.mark.parametrize("compute,eps", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_mfma_gaussian_error_bound(compute, eps):
    # Real data: the operand is rounded at four points (staged input and
    # collision sums, after MFMA passes 1, 2 and 3), each a relative error
    # <= eps of a quantity whose Walsh-Hadamard transform is taken; the
    # transform is an isometry up to sqrt(b), so the error of p is bounded
    # in norm by ~ 4 eps ||p||.  Checked elementwise with max |dp| <= 8 eps
    # max-norm-scaled, and the estimate within 8 eps ||C||_F / sqrt(d).
    announce(f"mfma {compute} gaussian error")
    w = small_random(256, 128, 200, 15, 3, seed=31)
    res = cmm.estimate(dev(w.A), dev(w.B), w.d, w.log2b, keys=w.keys, compute=compute)
    C, p_ref, t1, t2 = _ref(w, 256, 200)
    dp = np.abs(host(res.p) - p_ref)
    rms_p = np.sqrt(np.mean(p_ref ** 2))
    print(f"{compute}: max|dp|/rms(p) = {dp.max() / rms_p:.3e}, rms(dp)/rms(p) = "
          f"{np.sqrt(np.mean(dp ** 2)) / rms_p:.3e}", flush=True)
    assert np.sqrt(np.mean(dp ** 2)) <= 8 * eps * rms_p * np.sqrt(128)


def test_mfma_planted_8192_full_size():
    from workloads.metrics import planted_recall
    announce("mfma planted n=8192 b=2^18 d=9 bf16 + f16 + f64")
    w = planted_8192(0)
    A, B = dev(w.A), dev(w.B)
    t1, t2 = O.hash_tables(w.keys, w.n, w.n, w.log2b)
    p_ref = O.bucket_sums(O.product(w.A, w.B), t1, t2, w.log2b)
    rows = np.arange(0, w.n, 64)
    C_ref_rows = O.extract(p_ref, t1, t2, "median", rows=rows)
    for compute in ("f64", "f16", "bf16"):
        res = cmm.estimate(A, B, w.d, w.log2b, keys=w.keys, compute=compute)
        p = host(res.p)
        C_hat = host(res.C_hat)
        rel = np.max(np.abs(p - p_ref)) / np.max(np.abs(p_ref))
        rec = planted_recall(C_hat, w.rows, w.cols, w.tau)
        print(f"{compute}: max|dp|/max|p| = {rel:.3e}, recall {rec['recalled']}/{rec['planted']}",
              flush=True)
        if compute == "f64":
            # integer data below 2^53: exact
            assert np.array_equal(p, p_ref)
            assert np.array_equal(C_hat[rows], C_ref_rows)
        assert rec["recall"] >= 1.0 - 2.0 / rec["planted"]


@pytest.mark.parametrize("n", [10000, 12000])
@pytest.mark.parametrize("compute,eps", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_mfma_merged_chains_overflow(n, compute, eps):
    # At n = 10000 the two-row chains outnumber the sums the kernel can stage
    # beside a row (the rest take collision descriptors); at n = 12000 the
    # chains left to descriptors exceed their slots, so no chain is merged
    # ahead of the kernel.  Same error bound as the Gaussian case above.
    announce(f"mfma {compute} merged-chain overflow n={n}")
    rng = np.random.default_rng(n)
    n_inner, log2b, d = 16, 14, 3
    A = rng.standard_normal((n, n_inner))
    B = rng.standard_normal((n_inner, n))
    keys = draw_keys(d, 5 + n)
    from types import SimpleNamespace
    w = SimpleNamespace(A=A, B=B, keys=keys, log2b=log2b, d=d)
    res = cmm.estimate(dev(A), dev(B), d, log2b, keys=keys, compute=compute)
    C, p_ref, t1, t2 = _ref(w, n, n)
    dp = np.abs(host(res.p) - p_ref)
    rms_p = np.sqrt(np.mean(p_ref ** 2))
    print(f"{compute} n={n}: rms(dp)/rms(p) = {np.sqrt(np.mean(dp ** 2)) / rms_p:.3e}", flush=True)
    assert np.sqrt(np.mean(dp ** 2)) <= 8 * eps * rms_p * np.sqrt(n_inner)
