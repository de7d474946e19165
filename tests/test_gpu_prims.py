"""GPU parity of the primitive entry points against the CPU oracle.

Integer-valued inputs are exact in FP32, so max-plus products, argmax,
residuals and b-norms must match bit for bit.  Real-valued inputs: every
value operation is one correctly rounded FP32 operation on both sides, so
P, argmax, U and V match the FP32-value oracle bit for bit; the b-norm is an
FP64 sum in another order, within 1e-12 relative of it and within 1e-5
relative of the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2205_06619_amd import synth


def fp32_abs_bound(R, M, U, V):
    """Bound on |FP32-value result - FP64 result| of a b-norm: each observed
    cell takes a few correctly rounded FP32 operations (residual, add, max,
    subtract) on values of magnitude at most s, each off by <= 2^-24 s."""
    s = max(float(np.abs(R[M == 1]).max()), float(np.abs(U).max()), float(np.abs(V).max()))
    return 8.0 * int(M.sum()) * 2.0 ** -24 * 4 * s


pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (1, 7, 2), (9, 1, 3), (63, 65, 1), (64, 64, 3), (65, 129, 20),
          (130, 70, 5), (200, 300, 64)]


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2205_06619_amd import stmf
    return stmf


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _case(m, n, r, seed, integer):
    rng = np.random.default_rng(seed)
    if integer:
        U = rng.integers(0, 50, (m, r)).astype(np.float32)
        V = rng.integers(0, 50, (r, n)).astype(np.float32)
        R = rng.integers(0, 120, (m, n)).astype(np.float32)
    else:
        U = rng.normal(0, 1, (m, r)).astype(np.float32)
        V = rng.normal(0, 1, (r, n)).astype(np.float32)
        R = (rng.normal(0, 2, (m, n)) * np.exp(rng.normal(0, 0.5, (1, n)))).astype(np.float32)
    M = (rng.random((m, n)) >= 0.3).astype(np.uint8)
    M = synth.fix_empty_lines(M, rng)
    Rn = R.copy(); Rn[M == 0] = np.nan   # unobserved values must never be read
    return U, V, R, Rn, M


@pytest.mark.parametrize("m,n,r", SHAPES)
@pytest.mark.parametrize("integer", [True, False])
def test_maxplus_product(S, m, n, r, integer):
    print(f"maxplus m={m} n={n} r={r} int={integer}", flush=True)
    U, V, *_ = _case(m, n, r, 1, integer)
    P, A = S.stmf_maxplus_product(_t(U), _t(V))
    oP, oA = oracle.maxplus(U, V, "f32")
    np.testing.assert_array_equal(P.cpu().numpy(), oP)
    np.testing.assert_array_equal(A.cpu().numpy(), oA)


def test_maxplus_ties_take_lowest_index(S):
    U = np.zeros((70, 5), np.float32); V = np.zeros((5, 66), np.float32)
    V[3] = 1; V[4] = 1          # components 3 and 4 tie everywhere
    P, A = S.stmf_maxplus_product(_t(U), _t(V))
    assert np.all(A.cpu().numpy() == 3) and np.all(P.cpu().numpy() == 1)


@pytest.mark.parametrize("m,n,r", SHAPES)
@pytest.mark.parametrize("integer", [True, False])
def test_masked_error(S, m, n, r, integer):
    print(f"masked_error m={m} n={n} r={r} int={integer}", flush=True)
    U, V, R, Rn, M = _case(m, n, r, 2, integer)
    err, td = S.stmf_masked_error(_t(Rn), _t(M), _t(U), _t(V))
    e = float(err.cpu().numpy()[0]); td = td.cpu().numpy()
    e32, td32, _ = oracle.masked_error(R, M, U, V, "f32")
    e64, td64, _ = oracle.masked_error(R, M, U, V, "f64")
    if integer:
        assert e == e32 == e64
        np.testing.assert_array_equal(td, td32)
    else:
        assert e == pytest.approx(e32, rel=1e-12, abs=0)
        np.testing.assert_allclose(td, td32, rtol=1e-12, atol=0)
        assert e == pytest.approx(e64, rel=1e-5, abs=0)


@pytest.mark.parametrize("op", ["U", "V"])
@pytest.mark.parametrize("m,n,r", [(1, 5, 2), (6, 1, 1), (40, 70, 3), (65, 130, 7), (129, 64, 20)])
@pytest.mark.parametrize("integer", [True, False])
def test_update(S, op, m, n, r, integer):
    print(f"update_{op} m={m} n={n} r={r} int={integer}", flush=True)
    import torch
    U, V, R, Rn, M = _case(m, n, r, 3, integer)
    # start from residual-consistent V as the fit does
    for k in range(r):
        V = oracle.col_res(R, M, U, V, k, "f32")
    V = V.astype(np.float32)
    rng = np.random.default_rng(4)
    obs = np.argwhere(M == 1)
    for trial in range(3):
        i, j = obs[rng.integers(len(obs))]
        k = int(rng.integers(r))
        Ug, Vg = _t(U), _t(V)
        fn = S.stmf_update_U if op == "U" else S.stmf_update_V
        err, Ub, Vb = fn(_t(Rn), _t(M), Ug, Vg, i, j, k)
        oU, oV, oe, oUb, oVb, _ = oracle.update(op, R, M, U, V, i, j, k, "f32")
        np.testing.assert_array_equal(Ug.cpu().numpy(), oU)
        np.testing.assert_array_equal(Vg.cpu().numpy(), oV)
        np.testing.assert_array_equal(Ub.cpu().numpy(), oUb)
        np.testing.assert_array_equal(Vb.cpu().numpy(), oVb)
        e = float(err.cpu().numpy()[0])
        if integer:
            assert e == oe
        else:
            assert e == pytest.approx(oe, rel=1e-12, abs=0)
            _, _, e64, *_ = oracle.update(op, R, M, U, V, i, j, k, "f64")
            assert e == pytest.approx(e64, rel=1e-5, abs=fp32_abs_bound(R, M, U, V))
        U, V = oU, oV
        torch.cuda.synchronize()


def test_update_rejects_unobserved_cell(S):
    U, V, R, Rn, M = _case(8, 9, 2, 5, True)
    M[2, 3] = 0
    with pytest.raises(S.StmfError) as ex:
        S.stmf_update_U(_t(Rn), _t(M), _t(U), _t(V), 2, 3, 0)
    assert ex.value.status == S.STMF_EINVAL


@pytest.mark.parametrize("line", ["row", "col"])
@pytest.mark.parametrize("op", ["U", "V"])
def test_update_rejects_empty_line_before_writing(S, line, op):
    # a residual over a line with no observed cell is undefined: the update
    # calls refuse such a mask before launching anything (U, V untouched)
    U, V, R, Rn, M = _case(8, 9, 2, 5, True)
    if line == "row":
        M[4, :] = 0
    else:
        M[:, 6] = 0
    Ud, Vd = _t(U), _t(V)
    fn = S.stmf_update_U if op == "U" else S.stmf_update_V
    with pytest.raises(S.StmfError) as ex:
        fn(_t(Rn), _t(M), Ud, Vd, 0, 0, 1)
    assert ex.value.status == S.STMF_EEMPTY_LINE
    np.testing.assert_array_equal(Ud.cpu().numpy(), U)
    np.testing.assert_array_equal(Vd.cpu().numpy(), V)
