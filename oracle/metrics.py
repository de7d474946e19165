"""Completion-quality metrics of Sec. 3.6 in plain numpy FP64 (test
infrastructure only, like the rest of this package).

* RMSE over a set of cells: sqrt(mean of (R - U (x) V)^2), the product
  evaluated in FP64 from the FP32 factors (RMSE-A on the training cells,
  RMSE-P on the held-out cells).
* Distance correlation (Szekely, Rizzo and Bakirov, Ann. Statist. 35(6),
  2007), the V-statistic form: with a_kl = |x_k - x_l| and b_kl = |y_k - y_l|
  double-centred into A and B, dCov^2 = mean(A * B), dVar^2(x) = mean(A * A),
  dCor = sqrt(dCov^2 / sqrt(dVar^2(x) dVar^2(y))) (0 when a variance is 0).
  Written out with the full N x N matrices: only for the small N of the
  tests.  The paper applies DC to the original and the approximated values
  of the held-out cells.

Parity of the product's precision is unpinned against the paper (it fixes
none); the GPU forms the product in FP32 values, this module in FP64, which
the tests allow for in their tolerance.
"""
from __future__ import annotations

import numpy as np


def maxplus_f64(U, V):
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    return np.max(U[:, :, None] + V[None, :, :], axis=1)


def rmse(R, M, U, V):
    P = maxplus_f64(U, V)
    sel = np.asarray(M).astype(bool)
    d = np.asarray(R, np.float64)[sel] - P[sel]
    return float(np.sqrt(np.mean(d * d))) if d.size else 0.0


def _centred(x):
    a = np.abs(x[:, None] - x[None, :])
    return a - a.mean(axis=0)[None, :] - a.mean(axis=1)[:, None] + a.mean()


def dcor_terms(x, y):
    """(dCov^2, dVar^2(x), dVar^2(y), dCor) of two equal-length samples."""
    x = np.asarray(x, np.float64).ravel()
    y = np.asarray(y, np.float64).ravel()
    A, B = _centred(x), _centred(y)
    dcov2 = float(np.mean(A * B))
    vx, vy = float(np.mean(A * A)), float(np.mean(B * B))
    den = np.sqrt(vx * vy)
    dc = float(np.sqrt(max(dcov2, 0.0) / den)) if den > 0 else 0.0
    return dcov2, vx, vy, dc


def dcor(x, y):
    return dcor_terms(x, y)[3]


def row_terms(x, y, k):
    """Per-sample sums of sample k over all l: sum a_kl, sum b_kl,
    sum a_kl b_kl, sum a_kl^2, sum b_kl^2 (O(N) each)."""
    x = np.asarray(x, np.float64).ravel()
    y = np.asarray(y, np.float64).ravel()
    a = np.abs(x[k] - x)
    b = np.abs(y[k] - y)
    return np.array([a.sum(), b.sum(), (a * b).sum(), (a * a).sum(), (b * b).sum()])


def completion_metrics(R, M_train, M_test, U, V):
    """RMSE-A, RMSE-P and the DC of the held-out cells' (R, U (x) V) pairs,
    cells in row-major order."""
    P = maxplus_f64(U, V)
    sel = np.asarray(M_test).astype(bool)
    return {
        "rmse_a": rmse(R, M_train, U, V),
        "rmse_p": rmse(R, M_test, U, V),
        "dc": dcor(np.asarray(R, np.float64)[sel], P[sel]),
        "n_train": int(np.asarray(M_train).astype(bool).sum()),
        "n_test": int(sel.sum()),
    }
