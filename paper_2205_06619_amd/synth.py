"""Seeded synthetic inputs for sparse tropical matrix factorization.

This module only draws inputs: data matrices R, observation masks M and the
per-problem descriptors of the batched and serving workloads.  It holds none
of the factorization method's arithmetic and is shared by the tests, the
benchmark and the CPU oracle's callers, so that both sides of every parity
check see identical inputs.

Planted data is built as R = U* (x) V* (the max-plus product of Section 2 of
the paper) from seeded random factors; that construction is part of the input
recipe, not of the method, and is written here with plain numpy.

Workloads (all seeded, all synthetic):

* ``int_planted``   integer planted matrix, uniform ints in [0, 100], a fixed
                    number of cells masked out uniformly without replacement
                    (the exact-arithmetic case; every value < 2**24).
* ``gene_expr``     stand-in for a gene-expression matrix: planted rank-5
                    N(0,1) factors, N(0, 0.1) noise, per-column log-normal
                    scale exp(N(0, 0.5)), cells missing uniformly.
* ``large``         planted rank-20 U[0,10] factors plus N(0, 0.5) noise,
                    row-dependent missingness 0.4 + 0.6 * Beta(2,2).
* ``batched``       many problems of uneven shape, rank and missing fraction.

The paper's own experiments mask 20% of cells uniformly as a test set
(Section 3.7) and use synthetic R_lambda matrices (Section 3.4);
``r_lambda`` reproduces that recipe.
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np

__all__ = [
    "maxplus_planted",
    "fix_empty_lines",
    "int_planted",
    "gene_expr",
    "large",
    "r_lambda",
    "BatchProblem",
    "batched_problems",
    "poisson_arrivals",
    "tiny_int_case",
    "holdout",
]


def maxplus_planted(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Planted matrix A (x) B, built one rank component at a time (float32)."""
    A = np.asarray(A, dtype=np.float32)
    B = np.asarray(B, dtype=np.float32)
    out = np.add.outer(A[:, 0], B[0, :])
    for k in range(1, A.shape[1]):
        np.maximum(out, np.add.outer(A[:, k], B[k, :]), out=out)
    return out.astype(np.float32)


def fix_empty_lines(M: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Re-observe one random cell in every empty row and column (in place)."""
    m, n = M.shape
    for _ in range(4):
        rows = np.flatnonzero(M.sum(axis=1) == 0)
        for i in rows:
            M[i, rng.integers(0, n)] = 1
        cols = np.flatnonzero(M.sum(axis=0) == 0)
        for j in cols:
            M[rng.integers(0, m), j] = 1
        if not len(rows) and not len(cols):
            break
    return M


def _mask_exact(m: int, n: int, n_missing: int, rng) -> np.ndarray:
    M = np.ones(m * n, dtype=np.uint8)
    M[rng.choice(m * n, size=n_missing, replace=False)] = 0
    return fix_empty_lines(M.reshape(m, n), rng)


def _mask_uniform(m: int, n: int, p_missing: float, rng) -> np.ndarray:
    M = (rng.random((m, n)) >= p_missing).astype(np.uint8)
    return fix_empty_lines(M, rng)


def int_planted(m: int = 200, n: int = 100, rank: int = 3, missing: float = 0.2,
                seed: int = 0, hi: int = 100) -> Tuple[np.ndarray, np.ndarray]:
    """Integer planted data: U*, V* uniform ints in [0, hi]; R = U* (x) V*.

    Exactly round(missing * m * n) cells are masked out, drawn uniformly
    without replacement.  Every value is an integer < 2**24, so FP32 holds it
    exactly.
    """
    rng = np.random.default_rng(seed)
    U = rng.integers(0, hi + 1, size=(m, rank)).astype(np.float32)
    V = rng.integers(0, hi + 1, size=(rank, n)).astype(np.float32)
    R = maxplus_planted(U, V)
    M = _mask_exact(m, n, int(round(missing * m * n)), rng)
    return R, M


def gene_expr(m: int = 500, n: int = 2000, rank: int = 5, missing: float = 0.5,
              seed: int = 2) -> Tuple[np.ndarray, np.ndarray]:
    """Gene-expression-shaped real data (stand-in for the TCGA matrices).

    R = U* (x) V* + N(0, 0.1) with U*, V* ~ N(0, 1), then every column j is
    scaled by exp(z_j), z_j ~ N(0, 0.5) (log-normal per-column scale);
    cells are missing uniformly with probability ``missing``.
    """
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((m, rank)).astype(np.float32)
    V = rng.standard_normal((rank, n)).astype(np.float32)
    R = maxplus_planted(U, V).astype(np.float64)
    R += rng.normal(0.0, 0.1, size=(m, n))
    R *= np.exp(rng.normal(0.0, 0.5, size=(1, n)))
    M = _mask_uniform(m, n, missing, rng)
    return R.astype(np.float32), M


def large(m: int = 2000, n: int = 20000, rank: int = 20, seed: int = 3
          ) -> Tuple[np.ndarray, np.ndarray]:
    """Large planted real data with row-dependent missingness.

    U*, V* ~ U[0, 10], R = U* (x) V* + N(0, 0.5); row i is missing each cell
    with probability q_i = 0.4 + 0.6 * b_i, b_i ~ Beta(2, 2) (mean 0.7).
    """
    rng = np.random.default_rng(seed)
    U = rng.uniform(0.0, 10.0, size=(m, rank)).astype(np.float32)
    V = rng.uniform(0.0, 10.0, size=(rank, n)).astype(np.float32)
    R = maxplus_planted(U, V)
    R += rng.normal(0.0, 0.5, size=(m, n)).astype(np.float32)
    q = 0.4 + 0.6 * rng.beta(2.0, 2.0, size=(m, 1))
    M = (rng.random((m, n)) >= q).astype(np.uint8)
    M = fix_empty_lines(M, rng)
    return R.astype(np.float32), M


def r_lambda(m: int, n: int, lam: float, rank: int = 3, missing: float = 0.2,
             seed: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Section 3.4 recipe: R = lam * (A (x) B) + (1 - lam) * (A . B), A, B ~ U[0,1)."""
    rng = np.random.default_rng(seed)
    A = rng.random((m, rank))
    B = rng.random((rank, n))
    R = lam * maxplus_planted(A, B).astype(np.float64) + (1.0 - lam) * (A @ B)
    M = _mask_exact(m, n, int(round(missing * m * n)), rng)
    return R.astype(np.float32), M


@dataclasses.dataclass
class BatchProblem:
    pid: int
    m: int
    n: int
    rank: int
    missing: float
    integer: bool
    R: np.ndarray
    M: np.ndarray


def batched_problems(count: int = 256, seed: int = 4, integer: bool = True,
                     m_range=(50, 1000), n_range=(50, 5000), r_range=(2, 30),
                     miss_range=(0.2, 0.8), only=None) -> List[BatchProblem]:
    """Problems of uneven shape: m, n, rank uniform ints, missing ~ U[lo, hi].

    ``integer`` selects planted uniform-int data (exact arithmetic); otherwise
    planted U[0,10] factors with N(0, 0.5) noise.  ``only`` (problem ids)
    builds just those problems of the population, the same as in the whole.
    """
    rng = np.random.default_rng(seed)
    out = []
    for pid in range(count):
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        r = int(rng.integers(r_range[0], r_range[1] + 1))
        miss = float(rng.uniform(miss_range[0], miss_range[1]))
        if only is not None and pid not in only:
            continue
        sub = np.random.default_rng([seed, pid])
        if integer:
            U = sub.integers(0, 101, size=(m, r)).astype(np.float32)
            V = sub.integers(0, 101, size=(r, n)).astype(np.float32)
            R = maxplus_planted(U, V)
        else:
            U = sub.uniform(0.0, 10.0, size=(m, r)).astype(np.float32)
            V = sub.uniform(0.0, 10.0, size=(r, n)).astype(np.float32)
            R = maxplus_planted(U, V) + sub.normal(0.0, 0.5, size=(m, n)).astype(np.float32)
        M = _mask_uniform(m, n, miss, sub)
        out.append(BatchProblem(pid, m, n, r, miss, integer, R.astype(np.float32), M))
    return out


def poisson_arrivals(count: int, rate_per_s: float, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds, increasing) of a Poisson stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def tiny_int_case(m: int, n: int, rank: int, seed: int, hi: int = 4,
                  missing: float = 0.25, planted: bool = False):
    """Tiny integer matrix (values in [0, hi]) with a mask with no empty line."""
    rng = np.random.default_rng(seed)
    if planted:
        U = rng.integers(0, hi + 1, size=(m, rank)).astype(np.float32)
        V = rng.integers(0, hi + 1, size=(rank, n)).astype(np.float32)
        R = maxplus_planted(U, V)
    else:
        R = rng.integers(0, hi + 1, size=(m, n)).astype(np.float32)
    M = _mask_uniform(m, n, missing, rng)
    return R, M


def holdout(M: np.ndarray, frac: float = 0.2, seed: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Split the observed cells of M into training and held-out masks: about
    round(frac * |Omega|) cells, drawn uniformly, go to the held-out set, each
    only if its row and column keep a training cell (a fit needs every line
    observed).  Returns (M_train, M_test), disjoint, their union M."""
    rng = np.random.default_rng(seed)
    M = np.asarray(M).astype(np.uint8)
    train = M.copy()
    test = np.zeros_like(M)
    obs = np.flatnonzero(M.ravel())
    want = int(round(frac * obs.size))
    rows = train.sum(axis=1).astype(np.int64)
    cols = train.sum(axis=0).astype(np.int64)
    n = M.shape[1]
    taken = 0
    for q in rng.permutation(obs):
        if taken == want:
            break
        i, j = divmod(int(q), n)
        if rows[i] > 1 and cols[j] > 1:
            train[i, j] = 0
            test[i, j] = 1
            rows[i] -= 1
            cols[j] -= 1
            taken += 1
    return train, test

