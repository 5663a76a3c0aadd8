"""FP64 Euclidean distance map, its gradient and the stress loss (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Inputs are FP32 arrays (exactly what the GPU sees); every computation below
converts them to FP64 first, which is exact.  Loops run over rows in plain
Python; inside a row numpy evaluates the definition for every column at
once.  Nothing is blocked, fused or reordered beyond that.

Layouts (the ones the library writes):
* packed: cell (i, j), 0 <= j <= i < N, at index i(i+1)/2 + j;
* full:   an N x N row-major matrix where only j <= i is defined;
* strict: the problem without the diagonal (Sec. II-A, Eq. (10)): cell
  (i, j), 0 <= j < i < N, at index i(i-1)/2 + j.
"""
from __future__ import annotations

from typing import Callable, Sequence

import numpy as np


def tri(i: int) -> int:
    return i * (i + 1) // 2


def _as64(X: np.ndarray) -> np.ndarray:
    X = np.asarray(X)
    if X.ndim != 2:
        raise ValueError("X must be (N, d)")
    return X.astype(np.float64)


def edm64_row(X64: np.ndarray, i: int) -> np.ndarray:
    """Row i of the lower-triangular EDM: f(i, j) for j = 0..i, with
    f(i, j) = sqrt(sum_k (a_i^k - a_j^k)^2) (Sec. IV, Eq. (17))."""
    diff = X64[i][None, :] - X64[: i + 1]
    return np.sqrt(np.sum(diff * diff, axis=1))


def edm64_packed(X: np.ndarray) -> np.ndarray:
    """All cells j <= i, packed row-major: N(N+1)/2 FP64 values."""
    X64 = _as64(X)
    N = X64.shape[0]
    out = np.empty(tri(N), dtype=np.float64)
    for i in range(N):
        out[tri(i): tri(i) + i + 1] = edm64_row(X64, i)
    return out


def edm64_strict(X: np.ndarray) -> np.ndarray:
    """All cells j < i, packed row-major without the diagonal: N(N-1)/2
    FP64 values, cell (i, j) at i(i-1)/2 + j."""
    X64 = _as64(X)
    N = X64.shape[0]
    out = np.empty(N * (N - 1) // 2 if N > 0 else 0, dtype=np.float64)
    for i in range(1, N):
        start = i * (i - 1) // 2
        out[start: start + i] = edm64_row(X64, i)[:i]
    return out


def edm64_full(X: np.ndarray) -> np.ndarray:
    """N x N FP64 matrix with the lower triangle (diagonal included) filled
    and NaN above it (those cells are not part of the td-problem)."""
    X64 = _as64(X)
    N = X64.shape[0]
    out = np.full((N, N), np.nan, dtype=np.float64)
    for i in range(N):
        out[i, : i + 1] = edm64_row(X64, i)
    return out


def edm64_rows(X: np.ndarray, rows: Sequence[int]) -> list:
    """The given rows of the lower-triangular EDM (row i has i+1 entries)."""
    X64 = _as64(X)
    return [edm64_row(X64, int(i)) for i in rows]


def edm64_batched(X_cat: np.ndarray, point_off: Sequence[int]) -> np.ndarray:
    """Independent packed EDMs of the sets X_cat[point_off[s]:point_off[s+1]],
    concatenated in set order (offset of set s = sum over t < s of
    n_t(n_t+1)/2)."""
    parts = []
    for s in range(len(point_off) - 1):
        parts.append(edm64_packed(X_cat[point_off[s]: point_off[s + 1]]))
    if not parts:
        return np.empty(0, dtype=np.float64)
    return np.concatenate(parts)


def edm_backward64(X: np.ndarray, dD_packed: np.ndarray) -> np.ndarray:
    """Gradient of a scalar loss through the lower-triangular EDM.

    With D_ij = ||x_i - x_j|| for j < i and g_ij = dL/dD_ij,
        dL/dx_i = sum_{j<i} g_ij (x_i - x_j) / D_ij
                - sum_{k>i} g_ki (x_k - x_i) / D_ki,
    a term being 0 where D = 0 (the one-sided derivative chosen at
    coincident points).  Diagonal cells carry no gradient: D_ii = 0 for
    every X.  Written in gather form, one point at a time.
    """
    X64 = _as64(X)
    N, d = X64.shape
    g = np.asarray(dD_packed, dtype=np.float64)
    if g.shape[0] != tri(N):
        raise ValueError("dD must hold N(N+1)/2 packed cells")
    dX = np.zeros((N, d), dtype=np.float64)
    for i in range(N):
        # cells (i, j), j < i: row i of the packed triangle
        if i > 0:
            diff = X64[i][None, :] - X64[:i]
            D = np.sqrt(np.sum(diff * diff, axis=1))
            gij = g[tri(i): tri(i) + i]
            c = np.where(D > 0, gij / np.where(D > 0, D, 1.0), 0.0)
            dX[i] += np.sum(c[:, None] * diff, axis=0)
        # cells (k, i), k > i: column i of the triangle
        if i < N - 1:
            ks = np.arange(i + 1, N)
            diff = X64[ks] - X64[i][None, :]
            D = np.sqrt(np.sum(diff * diff, axis=1))
            gki = g[ks * (ks + 1) // 2 + i]
            c = np.where(D > 0, gki / np.where(D > 0, D, 1.0), 0.0)
            dX[i] -= np.sum(c[:, None] * diff, axis=0)
    return dX


def stress64(X: np.ndarray, delta_packed: np.ndarray):
    """Stress L = sum_{j<i} (D_ij - delta_ij)^2 and its cell gradient
    dL/dD_ij = 2 (D_ij - delta_ij) (0 on the diagonal, which is not part of
    the sum).  Returns (L, D_packed, dD_packed), all FP64."""
    D = edm64_packed(X)
    delta = np.asarray(delta_packed, dtype=np.float64)
    N = np.asarray(X).shape[0]
    offdiag = np.ones(tri(N), dtype=bool)
    diag_idx = np.array([tri(i) + i for i in range(N)], dtype=np.int64)
    offdiag[diag_idx] = False
    r = np.where(offdiag, D - delta, 0.0)
    return float(np.sum(r * r)), D, 2.0 * r


def stress_grad64(X: np.ndarray, delta_packed: np.ndarray):
    """(L, dL/dX) of the stress loss, FP64."""
    L, _, dD = stress64(X, delta_packed)
    return L, edm_backward64(X, dD)


def central_differences(f: Callable[[np.ndarray], float], X: np.ndarray,
                        h: float = 1e-6) -> np.ndarray:
    """Central finite differences of a scalar function of X (FP64)."""
    X64 = np.array(X, dtype=np.float64)
    G = np.zeros_like(X64)
    for idx in np.ndindex(*X64.shape):
        xp = X64.copy()
        xm = X64.copy()
        xp[idx] += h
        xm[idx] -= h
        G[idx] = (f(xp) - f(xm)) / (2.0 * h)
    return G


# ---------------------------------------------------------------------------
# BF16 Gram form: the error bound the GPU result is judged against
# ---------------------------------------------------------------------------

U32 = 2.0 ** -24   # unit roundoff of FP32 (round to nearest)
U_BF16 = 2.0 ** -8  # unit roundoff of BF16 (8-bit significand)


def gram_bound(norm_i, norm_j, D64, d: int, split: bool = False):
    """Largest |D_gpu - D| allowed for a pair that the Gram path did not
    recompute, given ||x_i||, ||x_j||, the FP64 distance D and the feature
    count d (arrays broadcast).  u denotes the BF16 unit roundoff, u32 the
    FP32 one.

    Terms, BF16 inputs (split = False):
    * BF16 rounding of the inputs: |x~ - x| <= u |x| per coordinate, so
      by the triangle inequality | ||x~-y~|| - ||x-y|| | <= u (||x||+||y||).
    * FP32 accumulation of n~_i + n~_j - 2 x~.y~ with d-term sums (products
      of BF16 values are exact in FP32): |G - G_exact| <= E with
      E = 2 (d + 4) u32 (||x||^2 + ||y||^2) (1 + u)^2, and the square
      root turns E into at most E / D_lower where D_lower is a lower bound of
      the BF16 distance (pairs above the threshold are far from 0).
    * the final square root and store: 2 ulp of D.

    Split inputs (split = True: x = hi + lo with hi = bf16(x) and
    lo = bf16(x - hi), the dot product taken as hi.hi' + hi.lo' + lo.hi'):
    * x - hi is exact in FP32 and |x - hi| <= u |x|, so
      |x - (hi + lo)| <= u |x - hi| <= u^2 |x|: the representation term
      becomes u^2 (||x||+||y||);
    * the dot product sums 3d exact products, and the dropped lo.lo' is at
      most ||lo|| ||lo'|| <= u^2 (1 + u)^2 ||x|| ||y||:
      E = 2 (3d + 4) u32 (||x||^2 + ||y||^2) (1 + u)^2
          + 2 u^2 (1 + u)^2 ||x|| ||y||.
    """
    norm_i = np.asarray(norm_i, dtype=np.float64)
    norm_j = np.asarray(norm_j, dtype=np.float64)
    D64 = np.asarray(D64, dtype=np.float64)
    u = U_BF16
    if split:
        rep = u * u * (norm_i + norm_j)
        E = (2.0 * (3 * d + 4) * U32 * (norm_i ** 2 + norm_j ** 2) * (1 + u) ** 2
             + 2.0 * u * u * (1 + u) ** 2 * norm_i * norm_j)
    else:
        rep = u * (norm_i + norm_j)
        E = 2.0 * (d + 4) * U32 * (norm_i ** 2 + norm_j ** 2) * (1 + u) ** 2
    D_lower = np.maximum(D64 - rep, 0.0)
    acc = np.where(D_lower > 0, E / np.where(D_lower > 0, D_lower, 1.0),
                   np.sqrt(E))
    acc = np.minimum(acc, np.sqrt(E))
    return rep + acc + 4.0 * U32 * D64


def fp32_rel_tol() -> float:
    """Per-cell relative tolerance for FP32 difference-form distances
    against the FP64 oracle (|D_gpu - D| <= tol * D, and D_gpu == 0 where
    D == 0)."""
    return 1e-6


__all__ = [
    "edm64_row", "edm64_packed", "edm64_full", "edm64_rows", "edm64_batched",
    "edm_backward64", "stress64", "stress_grad64", "central_differences",
    "gram_bound", "fp32_rel_tol", "tri",
]
