"""Differentiation form: the mean-over-d compressed product as a
``torch.autograd.Function``.

For fixed hash functions the mean estimate C_hat = (1/d) sum_t L_t(A B)
(Section 3.1: every repetition is an unbiased linear estimate of A B) is
bilinear in (A, B).  The forward pass is ``cmm_estimate`` with the mean
estimator; the backward pass is ``cmm_estimate_backward``, the library's
hand-written adjoint (bucket sums of the upstream gradient, its transform,
the transposed transforms and the transposed count sketch), run on the same
hash tables.  Both run in the library's HIP kernels.
"""
from __future__ import annotations

import torch

from . import (cmm_backward_workspace_size, cmm_estimate_backward, cmm_hash, estimate,
               keys_tensor, make_problem)


class CompressedMatmulMean(torch.autograd.Function):
    """C_hat = mean over d repetitions of the compressed estimate of A B."""

    @staticmethod
    def forward(ctx, A, B, tab1, tab2, d: int, log2b: int, compute: str):
        A = A.contiguous()
        B = B.contiguous()
        est = estimate(A, B, d, log2b, tab1=tab1, tab2=tab2, compute=compute,
                       estimator="mean")
        ctx.save_for_backward(A, B, tab1, tab2)
        ctx.d, ctx.log2b, ctx.compute = d, log2b, compute
        return est.C_hat

    @staticmethod
    def backward(ctx, W):
        A, B, tab1, tab2 = ctx.saved_tensors
        W = W.to(A.dtype).contiguous()
        dA = torch.empty_like(A)
        dB = torch.empty_like(B)
        pr = make_problem(A, B, ctx.d, ctx.log2b, tab1=tab1, tab2=tab2, compute=ctx.compute,
                          estimator="mean")
        nbytes = cmm_backward_workspace_size(pr)
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=A.device)
        cmm_estimate_backward(pr, W, dA, dB, ws, nbytes)
        return (dA if ctx.needs_input_grad[0] else None,
                dB if ctx.needs_input_grad[1] else None, None, None, None, None, None)


def hash_tables(keys, d: int, n_rows: int, n_cols: int, log2b: int, device="cuda"):
    """Tables (int32 device tensors with the uint32 bits) of the keys."""
    if not hasattr(keys, "data_ptr"):
        keys = keys_tensor(keys, device)
    tab1 = torch.empty((d, n_rows), dtype=torch.int32, device=device)
    tab2 = torch.empty((d, n_cols), dtype=torch.int32, device=device)
    cmm_hash(keys, d, n_rows, n_cols, log2b, tab1, tab2)
    return tab1, tab2


def compressed_matmul(A, B, d: int, log2b: int, *, keys=None, tab1=None, tab2=None,
                      compute: str = "f32"):
    """Differentiable mean-over-d compressed product of A and B.

    Give the hash ``keys`` (uint64[d][4][2]) or the tables ``tab1`` /
    ``tab2``; the backward pass uses the same tables as the forward pass."""
    if keys is not None:
        tab1, tab2 = hash_tables(keys, d, A.shape[0], B.shape[1], log2b, A.device)
    if tab1 is None or tab2 is None:
        raise ValueError("compressed_matmul needs keys or both tables")
    return CompressedMatmulMean.apply(A, B, tab1, tab2, d, log2b, compute)
