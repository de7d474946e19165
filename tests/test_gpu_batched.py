"""GPU tests of the batched path (stmf_fit_batched): many fits of uneven shape
and several restarts in one persistent launch (captured in a HIP graph),
whose groups of workgroups take fits from a device queue.  Batching changes
where a fit runs, never its arithmetic: every fit equals stmf_fit alone with
the restart's seed, bit for bit (integer and real data; a fit's result does
not depend on its group size), and on integer data equals the oracle."""
import numpy as np
import pytest

import oracle
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


def _problems(integer, count, seed):
    return synth.batched_problems(count, seed=seed, integer=integer, m_range=(12, 110),
                                  n_range=(12, 150), r_range=(2, 5), miss_range=(0.2, 0.6))


def _restart_seeds(seed, restarts):
    # one restart: the problem's seed; several: SplitMix64 outputs of it
    if restarts == 1:
        return [seed]
    return [int(x) for x in oracle.splitmix64(seed, restarts)]


def _group(gcap, m, n):
    # a fit's workgroups: the group size (0: no limit), at most its 64 x 64
    # tiles of the working orientation (fewer than the device holds at once)
    tiles = -(-min(m, n) // 64) * -(-max(m, n) // 64)
    return tiles if gcap == 0 else max(1, min(gcap, tiles))


def _dev(probs, iters):
    return [dict(R=_t(p.R), M=_t(p.M), rank=p.rank, iters=iters, seed=1000 + p.pid) for p in probs]


@pytest.mark.parametrize("gcap", [1, 0, 3])
@pytest.mark.parametrize("integer", [True, False])
def test_batched_equals_plain(S, integer, gcap):
    print(f"batched vs plain integer={integer} group={gcap}", flush=True)
    probs = _problems(integer, 6, seed=40 + int(integer))
    iters, restarts = 3, 2
    dev = _dev(probs, iters)
    outs, statuses, info = S.stmf_fit_batched(dev, restarts=restarts, group_size=gcap)
    assert statuses == [0] * len(probs)
    total_trials = 0
    for p, d, (U, V, T) in zip(probs, dev, outs):
        for q, sd in enumerate(_restart_seeds(d["seed"], restarts)):
            g = S.stmf_fit(d["R"], d["M"], p.rank, iters, seed=sd,
                           group_size=_group(gcap, p.m, p.n))
            total_trials += g.info["trials"]
            np.testing.assert_array_equal(U[q].cpu().numpy(), g.U.cpu().numpy())
            np.testing.assert_array_equal(V[q].cpu().numpy(), g.V.cpu().numpy())
            np.testing.assert_array_equal(T[q].cpu().numpy(), g.traj)
    assert info["trials"] == total_trials


def test_batched_integer_matches_oracle(S):
    print("batched integer vs oracle", flush=True)
    probs = _problems(True, 4, seed=47)
    iters, restarts = 2, 2
    dev = _dev(probs, iters)
    outs, statuses, _ = S.stmf_fit_batched(dev, restarts=restarts, integer_exact=1)
    assert statuses == [0] * len(probs)
    for p, d, (U, V, T) in zip(probs, dev, outs):
        for q, sd in enumerate(_restart_seeds(d["seed"], restarts)):
            o = oracle.fit(p.R, p.M, p.rank, iters, seed=sd, prec="f32")
            assert o.status == 0
            np.testing.assert_array_equal(U[q].cpu().numpy(), o.U)
            np.testing.assert_array_equal(V[q].cpu().numpy(), o.V)
            np.testing.assert_array_equal(T[q].cpu().numpy(), o.traj)


def test_batched_single_restart_uses_problem_seed(S):
    print("batched one restart", flush=True)
    probs = _problems(True, 3, seed=49)
    dev = _dev(probs, 2)
    outs, statuses, _ = S.stmf_fit_batched(dev, restarts=1)
    assert statuses == [0, 0, 0]
    for p, d, (U, V, T) in zip(probs, dev, outs):
        g = S.stmf_fit(d["R"], d["M"], p.rank, 2, seed=d["seed"])
        np.testing.assert_array_equal(U[0].cpu().numpy(), g.U.cpu().numpy())
        np.testing.assert_array_equal(T[0].cpu().numpy(), g.traj)


def test_batched_bad_problem_is_isolated(S):
    print("batched bad problem", flush=True)
    probs = _problems(True, 3, seed=48)
    dev = _dev(probs, 2)
    Mbad = probs[1].M.copy()
    Mbad[0, :] = 0  # an empty row
    dev[1]["M"] = _t(Mbad)
    outs, statuses, _ = S.stmf_fit_batched(dev, restarts=2)
    assert statuses[1] == S.STMF_EEMPTY_LINE
    assert statuses[0] == 0 and statuses[2] == 0
    for idx in (0, 2):
        p, d = probs[idx], dev[idx]
        sd = _restart_seeds(d["seed"], 2)[1]
        g = S.stmf_fit(d["R"], d["M"], p.rank, 2, seed=sd)
        np.testing.assert_array_equal(outs[idx][0][1].cpu().numpy(), g.U.cpu().numpy())


def test_batched_rejects_bad_arguments(S):
    print("batched arguments", flush=True)
    probs = _problems(True, 1, seed=50)
    dev = _dev(probs, 1)
    with pytest.raises(S.StmfError):
        S.stmf_fit_batched(dev, restarts=0)
    with pytest.raises(S.StmfError):
        S.stmf_fit_batched(dev, restarts=1, decision_log=1, log_cap=4)
    with pytest.raises(S.StmfError):
        S.stmf_fit_batched(dev, restarts=1, strategy=2)


def test_batched_row_visit_prefix_equals_plain_prefix(S):
    # max_row_visits stops every fit after that many row visits: each fit's
    # state then is the plain fit's after the same prefix
    print("batched prefix", flush=True)
    probs = _problems(False, 5, seed=56)
    dev = _dev(probs, 3)
    outs, statuses, info = S.stmf_fit_batched(dev, restarts=2, max_row_visits=7, init_mode=1)
    assert statuses == [0] * len(probs)
    for p, d, (U, V, T) in zip(probs, dev, outs):
        for q, sd in enumerate(_restart_seeds(d["seed"], 2)):
            g = S.stmf_fit(d["R"], d["M"], p.rank, 3, seed=sd, init_mode=1, max_row_visits=7)
            np.testing.assert_array_equal(U[q].cpu().numpy(), g.U.cpu().numpy())
            np.testing.assert_array_equal(V[q].cpu().numpy(), g.V.cpu().numpy())
            assert T[q].cpu().numpy()[0] == g.traj[0]


@pytest.mark.parametrize("gcap", [64, 0])
def test_batched_wide_fits_on_large_groups(S, gcap):
    # three fits of 4 x 66 tiles on groups of 64 workgroups (or the
    # library's choice), wider than one workgroup's column sort
    print(f"batched wide fits group={gcap}", flush=True)
    rng = np.random.default_rng(51)
    dev = []
    for q in range(3):
        R = rng.random((200, 4200)).astype(np.float32)
        M = (rng.random((200, 4200)) < 0.5).astype(np.uint8)
        M[:, 0] = 1
        M[0, :] = 1
        dev.append(dict(R=_t(R), M=_t(M), rank=2, iters=1, seed=60 + q))
    outs, statuses, info = S.stmf_fit_batched(dev, restarts=1, group_size=gcap)
    assert statuses == [0, 0, 0]
    if gcap:
        assert info["group_size"] == gcap
    for d, (U, V, T) in zip(dev, outs):
        g = S.stmf_fit(d["R"], d["M"], 2, 1, seed=d["seed"])
        assert g.info["group_size"] >= 64
        np.testing.assert_array_equal(U[0].cpu().numpy(), g.U.cpu().numpy())
        np.testing.assert_array_equal(V[0].cpu().numpy(), g.V.cpu().numpy())
        np.testing.assert_array_equal(T[0].cpu().numpy(), g.traj)


@pytest.mark.parametrize("gcap", [1, 0])
def test_batched_zero_passes_and_tiny_problems(S, gcap):
    # a fit of zero passes (its initial error only) and 1 x n / m x 1
    # problems beside ordinary ones, through the queue launch and the rounds
    print(f"batched edge problems group={gcap}", flush=True)
    probs = _problems(True, 3, seed=52)
    dev = _dev(probs, 2)
    dev[0]["iters"] = 0
    for shape, seed in (((1, 70), 53), ((90, 1), 54)):
        R, M = synth.int_planted(shape[0], shape[1], 1, 0.0, seed=seed)
        dev.append(dict(R=_t(R), M=_t(M), rank=1, iters=2, seed=seed))
    outs, statuses, _ = S.stmf_fit_batched(dev, restarts=2, group_size=gcap)
    assert statuses == [0] * len(dev)
    for d, (U, V, T) in zip(dev, outs):
        m, n = d["R"].shape
        for q, sd in enumerate(_restart_seeds(d["seed"], 2)):
            g = S.stmf_fit(d["R"], d["M"], d["rank"], d["iters"], seed=sd,
                           group_size=_group(gcap, m, n))
            np.testing.assert_array_equal(U[q].cpu().numpy(), g.U.cpu().numpy())
            np.testing.assert_array_equal(V[q].cpu().numpy(), g.V.cpu().numpy())
            np.testing.assert_array_equal(T[q].cpu().numpy(), g.traj)


@pytest.mark.parametrize("gcap", [8, 32])
def test_batched_more_fits_than_groups(S, gcap):
    # 20 problems x 4 restarts = 80 fits on groups of 8 (32 groups) or 32
    # (8 groups) workgroups: groups take several fits each from the queue
    print(f"batched 80 fits group={gcap}", flush=True)
    probs = synth.batched_problems(20, seed=55, integer=False, m_range=(40, 200),
                                   n_range=(60, 400), r_range=(2, 6), miss_range=(0.2, 0.7))
    dev = _dev(probs, 2)
    outs, statuses, info = S.stmf_fit_batched(dev, restarts=4, group_size=gcap, init_mode=1)
    assert statuses == [0] * len(probs)
    assert info["group_size"] == gcap
    for p, d, (U, V, T) in zip(probs, dev, outs):
        for q, sd in enumerate(_restart_seeds(d["seed"], 4)):
            g = S.stmf_fit(d["R"], d["M"], p.rank, 2, seed=sd, init_mode=1)
            np.testing.assert_array_equal(U[q].cpu().numpy(), g.U.cpu().numpy())
            np.testing.assert_array_equal(V[q].cpu().numpy(), g.V.cpu().numpy())
            np.testing.assert_array_equal(T[q].cpu().numpy(), g.traj)


@pytest.mark.timeout(600)
def test_batched_population_subset_matches_oracle(S):
    # the two smallest problems of the 256-problem batched population (integer
    # planted, seed 4): 68 x 247 rank 6 and 57 x 379 rank 11, each with its 8
    # restarts, one pass, batched: every one of the 16 fits equals the oracle
    # bit for bit
    print("batched population subset vs oracle", flush=True)
    probs = synth.batched_problems(256, seed=4, integer=True, only=(62, 73))
    assert sorted((p.m, p.n, p.rank) for p in probs) == [(57, 379, 11), (68, 247, 6)]
    dev = _dev(probs, 1)
    outs, statuses, _ = S.stmf_fit_batched(dev, restarts=8, integer_exact=1)
    assert statuses == [0, 0]
    for p, d, (U, V, T) in zip(probs, dev, outs):
        for q, sd in enumerate(_restart_seeds(d["seed"], 8)):
            o = oracle.fit(p.R, p.M, p.rank, 1, seed=sd, prec="f32", integer_exact=1)
            assert o.status == 0
            np.testing.assert_array_equal(U[q].cpu().numpy(), o.U)
            np.testing.assert_array_equal(V[q].cpu().numpy(), o.V)
            np.testing.assert_array_equal(T[q].cpu().numpy(), o.traj)
