"""GPU parity of the completion-quality metrics (Sec. 3.6) against the
oracle's numpy FP64 definitions, at sizes the oracle handles in full, and at
the paper's large synthetic size (10000 x 300, 20% held out: 600,000
held-out cells) through per-sample sums the oracle computes one by one and
through an exact factorization (RMSE 0, DC 1).

Tolerances: the distance correlation is FP64 on both sides (the GPU through
the expanded double-centring identity, the oracle through the matrices):
1e-9 relative.  The RMSEs and the DC of a fit's held-out cells differ by the
FP32 product on the GPU against an FP64 product in the oracle: 1e-5
relative, plus 2^-23 max|R| absolute for the RMSEs (half an ulp of the
product, the whole difference when the fit is exact)."""
import numpy as np
import pytest

from oracle import metrics
from paper_2205_06619_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2205_06619_amd import stmf
    return stmf


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("N", [0, 1, 2, 3, 255, 257, 2048, 2049, 3000])
def test_dcor_equals_oracle(S, N):
    print(f"dcor N={N}", flush=True)
    rng = np.random.default_rng(N)
    x = rng.standard_normal(N).astype(np.float32)
    y = (np.tanh(x) + 0.3 * rng.standard_normal(N)).astype(np.float32)
    g = S.stmf_distance_correlation(_t(x), _t(y))
    if N == 0:
        assert g == dict(dcor=0.0, dcov2=0.0, dvarx2=0.0, dvary2=0.0)
        return
    dcov2, vx, vy, dc = metrics.dcor_terms(x, y)
    if N == 1:
        assert g["dcor"] == 0.0 and dc == 0.0
        return
    np.testing.assert_allclose([g["dcov2"], g["dvarx2"], g["dvary2"], g["dcor"]],
                               [dcov2, vx, vy, dc], rtol=1e-9)


def test_dcor_hand_example(S):
    print("dcor 3-point", flush=True)
    g = S.stmf_distance_correlation(_t(np.array([0, 1, 2], np.float32)),
                                    _t(np.array([0, 1, 4], np.float32)))
    assert g["dcov2"] == pytest.approx(80 / 81, rel=1e-13)
    assert g["dcor"] ** 2 == pytest.approx(80 / np.sqrt(7360), rel=1e-12)


def test_dcor_row_terms_at_full_size(S):
    # the 600,000 held-out cells of a 10000 x 300 matrix: per-sample sums
    # sampled against the oracle, and the whole result against the same sums
    print("dcor N=600000 row terms", flush=True)
    rng = np.random.default_rng(11)
    N = 600_000
    x = rng.random(N).astype(np.float32)
    y = (x * x + 0.1 * rng.random(N)).astype(np.float32)
    g = S.stmf_distance_correlation(_t(x), _t(y), row_terms=True)
    T = g["row_terms"].cpu().numpy()
    for k in list(rng.integers(0, N, 12)) + [0, N - 1]:
        np.testing.assert_allclose(T[k], metrics.row_terms(x, y, int(k)), rtol=1e-10)
    # the final combination, restated in numpy from the GPU's own sums
    n = float(N)
    ra, rb = T[:, 0] / n, T[:, 1] / n
    ga, gb = T[:, 0].sum() / n ** 2, T[:, 1].sum() / n ** 2
    dcov2 = (T[:, 2].sum() - 2 * n * (ra * rb).sum() + n * n * ga * gb) / n ** 2
    assert g["dcov2"] == pytest.approx(dcov2, rel=1e-9)
    assert 0.9 < g["dcor"] <= 1.0


def test_completion_metrics_exact_factorization_full_size(S):
    # R = A (x) B at the paper's large synthetic size, 20% held out; the
    # planted factors reproduce every cell: RMSE-A = RMSE-P = 0, DC = 1
    print("quality exact 10000x300", flush=True)
    rng = np.random.default_rng(5)
    A = rng.random((10000, 3)).astype(np.float32)
    B = rng.random((3, 300)).astype(np.float32)
    R = synth.maxplus_planted(A, B)
    M = np.ones_like(R, np.uint8)
    tr, te = synth.holdout(M, 0.2, seed=5)
    g = S.stmf_completion_metrics(_t(R), _t(tr), _t(te), _t(A), _t(B))
    assert g["rmse_a"] == 0.0 and g["rmse_p"] == 0.0
    assert g["dc"] == pytest.approx(1.0, abs=1e-12)
    assert g["n_train"] == int(tr.sum()) and g["n_test"] == int(te.sum()) == 600_000


@pytest.mark.parametrize("lam", [0.0, 0.5, 1.0])
def test_quality_harness_equals_oracle_metrics(S, lam):
    # R_lambda (Sec. 3.4), 90 x 130, rank 3, 20% held out: the harness fits on
    # the training cells and measures; the oracle's metrics of the same
    # factors agree
    print(f"quality R_lambda lam={lam}", flush=True)
    from paper_2205_06619_amd import quality
    R, M = synth.r_lambda(90, 130, lam, rank=3, missing=0.0, seed=3)
    met, fit, (tr, te) = quality.evaluate(R, M, 3, 6, seed=3, split_seed=3, init_mode=1)
    o = metrics.completion_metrics(R, tr, te, fit.U.cpu().numpy(), fit.V.cpu().numpy())
    assert met["n_train"] == o["n_train"] and met["n_test"] == o["n_test"]
    # an FP32 product is within half an ulp of the FP64 one: an RMSE moves by
    # at most 2^-24 max|P|, which dominates when the fit is exact (lam = 1)
    tol = 2.0 ** -23 * float(np.abs(R).max())
    for key in ("rmse_a", "rmse_p"):
        assert met[key] == pytest.approx(o[key], rel=1e-5, abs=tol)
    assert met["dc"] == pytest.approx(o["dc"], rel=1e-5)
    assert 0.0 < met["dc"] <= 1.0
    # the training RMSE is that of the cells the fit minimised the b-norm over
    assert met["rmse_a"] <= np.sqrt(fit.traj[0] ** 2 / met["n_train"]) + 1e-6


def test_completion_metrics_overlapping_and_empty_sets(S):
    print("quality edge sets", flush=True)
    R, M = synth.r_lambda(20, 30, 0.5, rank=2, missing=0.0, seed=4)
    rng = np.random.default_rng(4)
    U = rng.random((20, 2)).astype(np.float32)
    V = rng.random((2, 30)).astype(np.float32)
    empty = np.zeros_like(M)
    g = S.stmf_completion_metrics(_t(R), _t(M), _t(empty), _t(U), _t(V))
    assert g["n_test"] == 0 and g["rmse_p"] == 0.0 and g["dc"] == 0.0
    o = metrics.rmse(R, M, U, V)
    assert g["rmse_a"] == pytest.approx(o, rel=1e-5)
    both = S.stmf_completion_metrics(_t(R), _t(M), _t(M), _t(U), _t(V))
    assert both["rmse_a"] == both["rmse_p"] == g["rmse_a"]
    assert both["dc"] == pytest.approx(metrics.dcor(R.ravel(), metrics.maxplus_f64(U, V).ravel()),
                                       rel=1e-5)
