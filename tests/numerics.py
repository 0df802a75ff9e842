"""Operand rounding to the reduced precisions, and the error tolerances
derived for the float32 and bf16 / fp16 paths (test infrastructure: no
arithmetic of the method itself).

Tolerance model.  Every kernel path computes, per repetition t, inner index
k and operand, a Walsh-Hadamard transform X = H x of a count sketch x
(Section 3.2), then p_hat = sum_k X o Y and p = 2^-m H p_hat.  A rounding
applied to the intermediate values after some butterfly levels is, under the
standard model, an independent error of standard deviation at most
u |v| / sqrt(3) on each intermediate value v (round to nearest, unit
roundoff u).  The levels that follow are +-1 combinations whose rows are
orthogonal, so one rounding level adds to each output X_u an error of
variance (u^2 / 3) sum over the intermediate values feeding X_u of |v|^2,
which is (u^2 / 3) ||x||_2^2 on average over u (the partial transform scales
the 2-norm by the square root of the number of values it combines, and
each output draws on that fraction of them).  With L levels:
    std(e^X_u) ~ u sqrt(L / 3) ||x||_2,   ||x||_2^2 ~ ||A[:, k]||_2^2.
The product term X o Y takes e^X Y + X e^Y; p_hat sums it over k, and the
inverse transform averages the b values of p_hat with +-1 weights, so
    std(dp) ~ u sqrt(2 L / 3) S / sqrt(b),  S^2 = sum_k ||A[:,k]||^2 ||B[k,:]||^2.
A float32 accumulation over runs of K values of k adds
u32 sqrt(K / 3) S / sqrt(b).  The elementwise tolerance is `sigmas` times
the sum; the median (or mean) over repetitions is 1-Lipschitz in the largest
deviation, so the same tolerance holds for C_hat.
"""
import numpy as np

U32 = 2.0 ** -24
U_BF16 = 2.0 ** -8
U_F16 = 2.0 ** -11


def round_f32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x) -> np.ndarray:
    """float64 -> float32 -> bf16, each round to nearest even (the operand
    copies the precision form makes)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def round_f16(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


def sketch_norm(A: np.ndarray, B: np.ndarray) -> float:
    """S = sqrt(sum_k ||A[:, k]||^2 ||B[k, :]||^2)."""
    a2 = np.sum(np.asarray(A, dtype=np.float64) ** 2, axis=0)
    b2 = np.sum(np.asarray(B, dtype=np.float64) ** 2, axis=1)
    return float(np.sqrt(np.sum(a2 * b2)))


def p_tolerance(A, B, log2b: int, u: float, levels: int, k_run: int, extra32: int = 0,
                sigmas: float = 8.0) -> float:
    """Elementwise tolerance on |p - p_ref| (and |C_hat - C_ref|): `levels`
    roundings of unit roundoff u in each transform, `extra32` more at the
    float32 unit roundoff (sums inside a matrix instruction), and float32
    accumulation over runs of `k_run` values of k."""
    s = sketch_norm(A, B)
    b = float(1 << log2b)
    std = (u * np.sqrt(2.0 * levels / 3.0) + U32 * np.sqrt(2.0 * extra32 / 3.0) +
           U32 * np.sqrt(k_run / 3.0)) * s / np.sqrt(b)
    return sigmas * std


def f32_tolerance(A, B, log2b: int, k_run: int, operands_rounded: bool = True,
                  sigmas: float = 8.0) -> float:
    """Float32 transform path: every butterfly level rounds (log2b levels
    plus the collision sums), accumulation in float32 over `k_run` values;
    one level more when the reference product is of the unrounded operands."""
    levels = log2b + 1 + (0 if operands_rounded else 1)
    return p_tolerance(A, B, log2b, U32, levels, k_run, sigmas=sigmas)
