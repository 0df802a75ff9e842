"""Heavy-hitter counters for an estimate C_hat (no estimator arithmetic).

The counters follow the correctness experiment of Section 5.4: big elements
above a threshold, small elements below it, and absolute-error hits.
"""
from __future__ import annotations

import numpy as np


def planted_recall(C_hat: np.ndarray, rows: np.ndarray, cols: np.ndarray, tau: float) -> dict:
    """Recall of planted entries with |C_hat| >= tau, plus background hits."""
    pairs = np.unique(rows.astype(np.int64) * C_hat.shape[1] + cols.astype(np.int64))
    flat = np.abs(C_hat).ravel()
    hit = flat[pairs] >= tau
    big = np.count_nonzero(flat >= tau)
    return {"planted": int(pairs.size), "recalled": int(hit.sum()),
            "recall": float(hit.mean()) if pairs.size else 1.0,
            "background_ge_tau": int(big - hit.sum()),
            "recalled_set": pairs[hit]}


def exact_recall(C_hat: np.ndarray, C_exact: np.ndarray, tol: float) -> dict:
    """Fraction of nonzeros of C recovered within ``tol``; zeros exceeding it."""
    nz = C_exact != 0
    ok = np.abs(C_hat - C_exact) <= tol
    return {"nonzeros": int(nz.sum()), "recovered": int((ok & nz).sum()),
            "recall": float((ok & nz).sum() / max(1, nz.sum())),
            "zero_wrong": int((~ok & ~nz).sum())}
