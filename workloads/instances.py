"""Instance families of the paper's evaluation (Section 5.2, Table 1).

Inputs only: these build A, B and the set of big entries; they hold none of
the method's arithmetic.  Written with torch so that the same recipe runs on
the CPU (tests, against the oracle) and on the GPU (the evaluation run);
the random streams of the two devices differ, so a seed names an instance
per device.  n must be a power of two.

Readings (the construction in Section 5.2 is partly garbled):

* LOGUNIT builds C = D1 D2 P from A = D1 Q, B = Q^-1 D2 P (the text's
  derivation multiplies D1 on the left).  D1 has floor(log2 n / 2) entries
  100, D2 ceil(log2 n / 2) entries 100 at other positions, both 0.01
  elsewhere, so C has log2 n entries 1 and n - log2 n entries 1e-4 (the
  text's 0.001 does not follow from its own construction).
* LOGUNIT and DIAGONAL need Q^-1; the paper draws Q uniformly in (-1, 1)
  and inverts it.  Here Q = H S (Sylvester Hadamard times a random sign
  diagonal), an orthogonal substitute with Q^-1 = Q^T / n exactly.  The
  estimate depends on the inputs only through C = A B (it is linear in
  each bucket sum of C), so the substitute changes rounding only.
* DIAGONAL: C = P D with |D_jj| uniform in [0.5, 1) and a random sign.
* COVARIANCE: entries N(0, 1/n) (the 1/n scale makes the planted entry
  about rho, as the text states), and b_j* = rho a_i* + sqrt(1 - rho^2)
  b~_j* (the text's sqrt(1 + rho^2) would not keep the column's variance).
* LIGHTBULB: entries +-1/sqrt(n); column j* of B is row i* of A with
  round(n (1 - rho) / 2) entries negated, so c_i*j* = 1 - 2 round(n (1 -
  rho) / 2) / n (0.80078 at n = 1024, rho = 0.8).
"""
from __future__ import annotations

import math
from types import SimpleNamespace

FAMILIES = ("logunit", "diagonal", "covariance", "lightbulb")


def _torch():
    import torch
    return torch


def _gen(seed: int, device):
    g = _torch().Generator(device=device)
    g.manual_seed(seed)
    return g


def _hadamard(n: int, device):
    torch = _torch()
    h = torch.ones((1, 1), dtype=torch.float64, device=device)
    while h.shape[0] < n:
        h = torch.cat([torch.cat([h, h], 1), torch.cat([h, -h], 1)], 0)
    return h


def _signs(n: int, g, device):
    torch = _torch()
    return torch.randint(0, 2, (n,), generator=g, device=device).to(torch.float64) * 2 - 1


def _check_n(n: int):
    if n < 2 or n & (n - 1):
        raise ValueError("instances need n a power of two >= 2")


def logunit(n: int, seed: int, device="cpu") -> SimpleNamespace:
    _check_n(n)
    torch = _torch()
    g = _gen(seed, device)
    L = int(math.log2(n))
    pos = torch.randperm(n, generator=g, device=device)
    d1 = torch.full((n,), 0.01, dtype=torch.float64, device=device)
    d2 = torch.full((n,), 0.01, dtype=torch.float64, device=device)
    d1[pos[:L // 2]] = 100.0
    d2[pos[L // 2:L]] = 100.0
    perm = torch.randperm(n, generator=g, device=device)
    s = _signs(n, g, device)
    H = _hadamard(n, device)
    A = d1[:, None] * H * s[None, :]                      # D1 Q
    B = torch.empty_like(A)
    B[:, perm] = (s[:, None] * H * d2[None, :]) / n        # Q^T D2 P / n
    big = pos[:L]
    return SimpleNamespace(name="logunit", n=n, A=A, B=B, big_rows=big, big_cols=perm[big],
                           C_rows=torch.arange(n, device=device), C_cols=perm, C_vals=d1 * d2)


def diagonal(n: int, seed: int, device="cpu") -> SimpleNamespace:
    _check_n(n)
    torch = _torch()
    g = _gen(seed, device)
    perm = torch.randperm(n, generator=g, device=device)
    mag = 0.5 + 0.5 * torch.rand(n, generator=g, dtype=torch.float64, device=device)
    v = mag * _signs(n, g, device)                         # C[m, perm[m]] = v[m]
    s = _signs(n, g, device)
    H = _hadamard(n, device)
    A = H * s[None, :]                                     # Q
    B = torch.empty_like(A)
    B[:, perm] = (s[:, None] * H * v[None, :]) / n         # Q^T P D / n
    rows = torch.arange(n, device=device)
    return SimpleNamespace(name="diagonal", n=n, A=A, B=B, big_rows=rows, big_cols=perm,
                           C_rows=rows, C_cols=perm, C_vals=v)


def covariance(n: int, seed: int, device="cpu", rho: float = 0.8) -> SimpleNamespace:
    _check_n(n)
    torch = _torch()
    g = _gen(seed, device)
    A = torch.randn((n, n), generator=g, dtype=torch.float64, device=device) / math.sqrt(n)
    B = torch.randn((n, n), generator=g, dtype=torch.float64, device=device) / math.sqrt(n)
    ij = torch.randint(0, n, (2,), generator=g, device=device)
    i, j = int(ij[0]), int(ij[1])
    B[:, j] = rho * A[i, :] + math.sqrt(1.0 - rho * rho) * B[:, j]
    return SimpleNamespace(name="covariance", n=n, A=A, B=B,
                           big_rows=torch.tensor([i], device=device),
                           big_cols=torch.tensor([j], device=device))


def lightbulb(n: int, seed: int, device="cpu", rho: float = 0.8) -> SimpleNamespace:
    _check_n(n)
    torch = _torch()
    g = _gen(seed, device)
    A = _signs(n * n, g, device).reshape(n, n) / math.sqrt(n)
    B = _signs(n * n, g, device).reshape(n, n) / math.sqrt(n)
    ij = torch.randint(0, n, (2,), generator=g, device=device)
    i, j = int(ij[0]), int(ij[1])
    flips = torch.randperm(n, generator=g, device=device)[:round(n * (1.0 - rho) / 2)]
    col = A[i, :].clone()
    col[flips] = -col[flips]
    B[:, j] = col
    return SimpleNamespace(name="lightbulb", n=n, A=A, B=B,
                           big_rows=torch.tensor([i], device=device),
                           big_cols=torch.tensor([j], device=device))


def instance(family: str, n: int, seed: int, device="cpu") -> SimpleNamespace:
    return {"logunit": logunit, "diagonal": diagonal, "covariance": covariance,
            "lightbulb": lightbulb}[family](n, seed, device)


def params(n: int, c_d: float, c_b: float) -> tuple[int, int]:
    """Section 5.6: d = 2 floor(c_d log2 n / 2) + 1 and b = c_b n, returned
    as (d, log2 b) with b rounded up to a power of two."""
    d = 2 * int(math.floor(c_d * math.log2(n) / 2)) + 1
    return d, max(1, math.ceil(math.log2(c_b * n)))
