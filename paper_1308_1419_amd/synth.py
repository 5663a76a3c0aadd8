"""Seeded synthetic inputs for the triangular-domain EDM workloads.

This module only draws random numbers; it holds none of the distance
arithmetic.  Both the GPU path and the CPU oracle are fed from here, so the
two see identical FP32 bits.  All generators use numpy's PCG64.

The paper names no dataset for its EDM experiments (Sec. IV); the workloads
below are synthetic stand-ins with the shapes the benchmarks use:

* ``uniform_points``   -- N points, d features, FP32 U[0, 1).
* ``gaussian_with_near_duplicates`` -- FP32 N(0, 1) points where a seeded 1%
  of them are replaced by a copy of another (non-replaced) point plus
  N(0, jitter^2) per coordinate, planting that many near-zero distances.
* ``stress_inputs``    -- X ~ U[0, 1) and X' = X + N(0, sigma^2).
* ``batched_sets``     -- S independent sets with sizes drawn uniformly from
  the inclusive integer range [n_min, n_max], concatenated.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

SEED_BASE = 1308141900


def workload_seed(index: int) -> int:
    return SEED_BASE + index


def uniform_points(N: int, d: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random((N, d), dtype=np.float32)


def gaussian_with_near_duplicates(N: int, d: int, seed: int, frac: float = 0.01,
                                  jitter: float = 1e-4
                                  ) -> Tuple[np.ndarray, np.ndarray]:
    """Returns (X, pairs) where pairs[t] = (copy, source) lists the planted
    near-duplicates (indices into X)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.standard_normal((N, d), dtype=np.float32)
    n_dup = int(frac * N)
    if n_dup == 0 or N < 2:
        return X, np.zeros((0, 2), dtype=np.int64)
    perm = rng.permutation(N)
    copies = np.sort(perm[:n_dup])
    keep = perm[n_dup:]
    sources = keep[rng.integers(0, len(keep), size=n_dup)]
    noise = rng.standard_normal((n_dup, d), dtype=np.float32) * np.float32(jitter)
    X[copies] = X[sources] + noise
    return X, np.stack([copies, sources], axis=1).astype(np.int64)


def stress_inputs(N: int, d: int, seed: int, sigma: float = 0.05
                  ) -> Tuple[np.ndarray, np.ndarray]:
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.random((N, d), dtype=np.float32)
    Xp = X + rng.standard_normal((N, d), dtype=np.float32) * np.float32(sigma)
    return X, Xp.astype(np.float32)


def batched_sets(num_sets: int, n_min: int, n_max: int, d: int, seed: int
                 ) -> Dict[str, np.ndarray]:
    """Concatenated point sets.  ``point_off[s]`` is the first point of set s
    (length num_sets+1) and ``out_off[s]`` the first packed output cell of set
    s, the running sum of n_t(n_t+1)/2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(n_min, n_max, size=num_sets, endpoint=True).astype(np.int64)
    point_off = np.zeros(num_sets + 1, dtype=np.int64)
    np.cumsum(sizes, out=point_off[1:])
    out_off = np.zeros(num_sets + 1, dtype=np.int64)
    np.cumsum(sizes * (sizes + 1) // 2, out=out_off[1:])
    X = rng.random((int(point_off[-1]), d), dtype=np.float32)
    return {"X": X, "sizes": sizes, "point_off": point_off, "out_off": out_off}


# The benchmark workloads (sizes and recipes), by name.
WORKLOADS: Dict[str, dict] = {
    "edm_n1024_d3_full": dict(index=1, N=1024, d=3, layout="full"),
    "edm_n30000_d3_full": dict(index=2, N=30000, d=3, layout="full"),
    "gram_n100000_d64_packed": dict(index=3, N=100000, d=64, layout="packed"),
    "stress_n20000_d3": dict(index=4, N=20000, d=3, layout="packed"),
    "batched_s4096_n64_4096_d3": dict(index=5, num_sets=4096, n_min=64,
                                      n_max=4096, d=3, layout="packed"),
}


def sample_rows(N: int, count: int, seed: int) -> List[int]:
    """A seeded sample of distinct row indices, always including the first
    and last rows."""
    rng = np.random.Generator(np.random.PCG64(seed))
    count = min(count, N)
    rows = set(rng.choice(N, size=count, replace=False).tolist())
    rows.update({0, N - 1})
    return sorted(rows)
