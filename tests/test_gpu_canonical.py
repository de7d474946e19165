"""A fit's result does not depend on how many workgroups share it.

The FP64 error of every trial is summed per tile, then over chunks of
consecutive tiles and a pairwise tree over the chunks: an order fixed by the
working shape alone.  One real-valued fit (where the summation order shows in
the low bits of every error, and through near-ties in the decisions) is run
at group sizes 1, 3, 5 and the library's own choice, through stmf_fit,
stmf_fit_batched and the serving engine; U, V and the trajectory must be
identical bit for bit."""
import numpy as np
import pytest

from paper_2205_06619_amd import synth

pytestmark = pytest.mark.gpu

M_, N_, RANK, ITERS, SEED = 150, 420, 4, 6, 31   # 3 x 7 = 21 tiles


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2205_06619_amd import stmf
    return stmf


@pytest.fixture(scope="module")
def case(S):
    import torch
    R, M = synth.gene_expr(M_, N_, RANK, 0.5, seed=SEED)
    Rd, Md = torch.from_numpy(R).cuda(), torch.from_numpy(M).cuda()
    ref = S.stmf_fit(Rd, Md, RANK, ITERS, seed=SEED, init_mode=1)
    assert ref.info["group_size"] == 21
    return Rd, Md, ref


def _same(U, V, traj, ref):
    np.testing.assert_array_equal(U.cpu().numpy(), ref.U.cpu().numpy())
    np.testing.assert_array_equal(V.cpu().numpy(), ref.V.cpu().numpy())
    np.testing.assert_array_equal(np.asarray(traj), ref.traj)


@pytest.mark.parametrize("G", [1, 3, 5])
def test_plain_fit_on_any_group_size(S, case, G):
    print(f"canonical: stmf_fit group {G}", flush=True)
    Rd, Md, ref = case
    g = S.stmf_fit(Rd, Md, RANK, ITERS, seed=SEED, init_mode=1, group_size=G)
    assert g.info["group_size"] == G
    _same(g.U, g.V, g.traj, ref)


@pytest.mark.parametrize("G", [1, 3, 0])
def test_batched_fit_on_any_group_size(S, case, G):
    print(f"canonical: stmf_fit_batched group {G}", flush=True)
    Rd, Md, ref = case
    outs, statuses, _ = S.stmf_fit_batched(
        [dict(R=Rd, M=Md, rank=RANK, iters=ITERS, seed=SEED)], restarts=1, init_mode=1,
        group_size=G)
    assert statuses == [0]
    U, V, T = outs[0]
    _same(U[0], V[0], T[0].cpu().numpy(), ref)


@pytest.mark.parametrize("G", [1, 3, 0])
def test_served_fit_on_any_group_size(S, case, G):
    print(f"canonical: engine group {G}", flush=True)
    Rd, Md, ref = case
    eng = S.stmf_engine_create(256 << 20, 4, group_size=G, init_mode=1)
    try:
        slot = S.stmf_engine_admit(eng, Rd, Md, RANK, ITERS, SEED)
        assert slot is not None
        for _ in range(100000):
            S.stmf_batch_tick(eng, 7)
            if S.stmf_engine_poll(eng, slot):
                break
        res = S.stmf_engine_retire(eng, slot)
    finally:
        S.stmf_engine_destroy(eng)
    _same(res.U, res.V, res.traj, ref)
