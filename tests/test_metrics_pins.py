"""Pins of the completion-quality metrics (Sec. 3.6) of the oracle and of the
held-out split: a hand-derived distance correlation (tests/golden), the
closed form of the population distance correlation of a bivariate normal
(Szekely, Rizzo, Bakirov 2007, Theorem 7), exact linear relations,
invariances, and RMSE special cases."""
import math

import numpy as np
import pytest

from oracle import metrics
from paper_2205_06619_amd import synth
from conftest import read_golden


def test_dcor_hand_derived_three_points():
    g = read_golden("dc_hand_3pt.txt")
    x = [float(v) for v in g["x"][0]]
    y = [float(v) for v in g["y"][0]]
    dcov2, vx, vy, dc = metrics.dcor_terms(x, y)
    def frac(key):
        num, den = g[key][0][0].split("/")
        return float(num) / float(den)
    assert dcov2 == pytest.approx(frac("dcov2"), rel=1e-14)
    assert vx == pytest.approx(frac("dvarx2"), rel=1e-14)
    assert vy == pytest.approx(frac("dvary2"), rel=1e-14)
    num, den = g["dcor2"][0][0].split("/")
    want = float(num) / math.sqrt(float(den[len("sqrt("):-1]))
    assert dc * dc == pytest.approx(want, rel=1e-13)


def _population_dcor_normal(rho):
    # Theorem 7 of Szekely, Rizzo, Bakirov (2007): bivariate normal, |rho| <= 1
    r = abs(rho)
    num = r * math.asin(r) + math.sqrt(1 - r * r) - r * math.asin(r / 2) - math.sqrt(4 - r * r) + 1
    den = 1 + math.pi / 3 - math.sqrt(3)
    return math.sqrt(num / den)


@pytest.mark.parametrize("rho", [0.0, 0.3, 0.7, 0.95])
def test_dcor_bivariate_normal_closed_form(rho):
    rng = np.random.default_rng(int(rho * 100) + 7)
    n = 2500
    z = rng.standard_normal((n, 2))
    x = z[:, 0]
    y = rho * z[:, 0] + math.sqrt(1 - rho * rho) * z[:, 1]
    got = metrics.dcor(x, y)
    # the V-statistic is biased upwards by O(N^-1/2) at independence
    assert abs(got - _population_dcor_normal(rho)) < 0.05


def test_dcor_exact_linear_relations_and_invariances():
    rng = np.random.default_rng(1)
    x = rng.random(300)
    for a, b in ((0.0, 2.0), (5.0, -0.5), (-3.0, 1e-3)):
        assert metrics.dcor(x, a + b * x) == pytest.approx(1.0, abs=1e-12)
    y = np.sin(7 * x) + 0.1 * rng.random(300)
    base = metrics.dcor(x, y)
    assert 0.0 < base < 1.0
    assert metrics.dcor(3.0 - 2.0 * x, 10.0 + 0.25 * y) == pytest.approx(base, rel=1e-12)
    assert metrics.dcor(y, x) == pytest.approx(base, rel=1e-12)
    assert metrics.dcor(x, np.full(300, 4.0)) == 0.0


def test_row_terms_add_up_to_the_matrix_sums():
    rng = np.random.default_rng(2)
    x, y = rng.random(50), rng.random(50)
    T = np.array([metrics.row_terms(x, y, k) for k in range(50)])
    a = np.abs(x[:, None] - x[None, :]); b = np.abs(y[:, None] - y[None, :])
    np.testing.assert_allclose(T.sum(axis=0), [a.sum(), b.sum(), (a * b).sum(), (a * a).sum(),
                                               (b * b).sum()], rtol=1e-12)


def test_rmse_special_cases():
    rng = np.random.default_rng(3)
    U = rng.integers(0, 9, (6, 2)).astype(np.float32)
    V = rng.integers(0, 9, (2, 7)).astype(np.float32)
    R = synth.maxplus_planted(U, V)
    M = np.ones_like(R, np.uint8)
    assert metrics.rmse(R, M, U, V) == 0.0
    assert metrics.rmse(R + 2.5, M, U, V) == pytest.approx(2.5, rel=1e-15)
    # one wrong cell of 5 observed: error 3 -> sqrt(9 / 5)
    M2 = np.zeros_like(M); M2[0, :5] = 1
    R2 = R.copy(); R2[0, 2] += 3
    assert metrics.rmse(R2, M2, U, V) == pytest.approx(math.sqrt(9 / 5), rel=1e-15)


@pytest.mark.parametrize("seed", [0, 1])
def test_holdout_split(seed):
    R, M = synth.r_lambda(60, 80, 0.5, seed=seed)
    tr, te = synth.holdout(M, 0.2, seed=seed)
    assert not np.any(tr & te)
    np.testing.assert_array_equal(tr | te, M)
    assert te.sum() == round(0.2 * M.sum())
    assert tr.sum(axis=1).min() >= 1 and tr.sum(axis=0).min() >= 1
    tr2, te2 = synth.holdout(M, 0.2, seed=seed)
    np.testing.assert_array_equal(te, te2)
