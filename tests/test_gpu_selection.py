"""GPU parity of the other ByRow selections (TD, TD_B, SEQ; Sec. 3.2.1), the
ByElement strategy (Sec. 3.2.2) and the row and column orders (PermR, PermC,
none; Sec. 3.3) against the CPU oracle.

As for TD_A: on integer data U, V, the trajectory and the decision log are
identical; on real data the values and decisions match and the trajectory
agrees within 1e-9 relative.  Shapes span several 64 x 64 tiles with ragged
tails, tall inputs (transposed working matrix), matrices wider than one
workgroup's sort (TD's row order through device memory), and cooperative
groups of several workgroups.
"""
import numpy as np
import pytest

import oracle
from paper_2205_06619_amd import synth

pytestmark = pytest.mark.gpu

SEL = {"TD_A": 0, "TD": 1, "TD_B": 2, "SEQ": 3}


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2205_06619_amd import stmf
    return stmf


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _log_rows(log):
    return [(int(r["iter"]), int(r["row"]), int(r["trials"]), int(r["noops"]), int(r["j"]),
             int(r["k"]), int(r["op"])) for r in log]


def _compare(g, o, exact=True):
    assert _log_rows(g.log) == _log_rows(o.log)
    if exact:
        np.testing.assert_array_equal(g.traj, o.traj)
        np.testing.assert_array_equal(g.log["e"], o.log["e"])
    else:
        np.testing.assert_allclose(g.traj, o.traj, rtol=1e-9, atol=0)
    np.testing.assert_array_equal(g.U.cpu().numpy(), o.U)
    np.testing.assert_array_equal(g.V.cpu().numpy(), o.V)
    assert g.info["trials"] == o.stats["trials"]
    assert g.info["noops"] == o.stats["noops"]
    assert g.info["accepted"] == o.stats["accepted"]


CASES = [  # m, n, rank, iters, seed, missing
    (60, 90, 3, 3, 1, 0.2), (70, 150, 4, 2, 2, 0.4), (150, 70, 2, 2, 3, 0.3),
    (1, 40, 2, 2, 4, 0.2), (33, 65, 1, 2, 5, 0.0),
]


@pytest.mark.parametrize("sel", ["TD", "TD_B", "SEQ"])
@pytest.mark.parametrize("m,n,rank,iters,seed,miss", CASES)
@pytest.mark.parametrize("group", [0, 1])
def test_selection_integer(S, sel, m, n, rank, iters, seed, miss, group):
    print(f"selection {sel} int {m}x{n} r={rank} group={group}", flush=True)
    R, M = synth.int_planted(m, n, rank, miss, seed=seed, hi=30)
    o = oracle.fit(R, M, rank, iters, seed=seed, prec="f32", init_hi=30, selection=SEL[sel])
    assert o.status == 0
    g = S.stmf_fit(_t(R), _t(M), rank, iters, seed=seed, init_hi=30.0, group_size=group,
                   selection=SEL[sel], log_cap=min(m, n) * iters + 1)
    _compare(g, o)
    assert o.stats["accepted"] > 0 or min(m, n) == 1


@pytest.mark.parametrize("sel", ["TD_A", "TD", "TD_B", "SEQ"])
@pytest.mark.parametrize("perm_mode", [1, 2])
def test_row_orders(S, sel, perm_mode):
    print(f"row order {perm_mode} {sel}", flush=True)
    R, M = synth.int_planted(48, 80, 3, 0.3, seed=11, hi=40)
    R[7] = R[20]; M[7] = M[20]  # two rows with the same minimum
    o = oracle.fit(R, M, 3, 3, seed=11, prec="f32", init_hi=40, selection=SEL[sel],
                   perm_mode=perm_mode)
    g = S.stmf_fit(_t(R), _t(M), 3, 3, seed=11, init_hi=40.0, selection=SEL[sel],
                   perm_mode=perm_mode, log_cap=200)
    _compare(g, o)


@pytest.mark.parametrize("group", [0, 1])
def test_permr_transposed(S, group):
    print(f"PermR tall group={group}", flush=True)
    R, M = synth.int_planted(130, 66, 2, 0.3, seed=12, hi=25)
    o = oracle.fit(R, M, 2, 2, seed=12, prec="f32", init_hi=25, perm_mode=1)
    g = S.stmf_fit(_t(R), _t(M), 2, 2, seed=12, init_hi=25.0, perm_mode=1, group_size=group,
                   log_cap=200)
    _compare(g, o)


@pytest.mark.parametrize("sel", ["TD", "TD_B", "SEQ"])
def test_selection_real(S, sel):
    print(f"selection {sel} real 60x150", flush=True)
    R, M = synth.gene_expr(60, 150, 4, 0.5, seed=2)
    o = oracle.fit(R, M, 4, 3, seed=2, prec="f32", init_mode=1, selection=SEL[sel])
    g = S.stmf_fit(_t(R), _t(M), 4, 3, seed=2, init_mode=1, selection=SEL[sel], log_cap=200)
    _compare(g, o, exact=False)


@pytest.mark.parametrize("group", [0, 1])
def test_td_wider_than_one_sort(S, group):
    # n > 4096: TD's row order and TD_A's column order go through device memory
    print(f"TD wide 12x4500 group={group}", flush=True)
    R, M = synth.int_planted(12, 4500, 2, 0.3, seed=13, hi=50)
    for sel in ("TD", "TD_A"):
        o = oracle.fit(R, M, 2, 1, seed=13, prec="f32", init_hi=50, selection=SEL[sel])
        g = S.stmf_fit(_t(R), _t(M), 2, 1, seed=13, init_hi=50.0, group_size=group,
                       selection=SEL[sel], log_cap=40)
        _compare(g, o)


@pytest.mark.parametrize("sel", ["TD", "TD_B"])
def test_selection_gene_expression_prefix(S, sel):
    # the full gene-expression-shaped workload (500 x 2000, rank 5, 50%
    # missing, Random Acol) in the cooperative launch: the first 12 row
    # visits, decision by decision
    print(f"selection {sel} real 500x2000 prefix", flush=True)
    R, M = synth.gene_expr()
    o = oracle.fit(R, M, 5, 50, seed=2, prec="f32", init_mode=1, row_limit=12, selection=SEL[sel])
    g = S.stmf_fit(_t(R), _t(M), 5, 50, seed=2, init_mode=1, max_row_visits=12, log_cap=64,
                   selection=SEL[sel])
    assert _log_rows(g.log) == _log_rows(o.log)
    np.testing.assert_allclose(g.log["e"], o.log["e"], rtol=1e-9)


def test_seq_prefix_larger(S):
    # SEQ evaluates every (j, k, operation) of a row: 100 x 400, rank 5, the
    # first 3 row visits (about 2000 trials each) in the cooperative launch
    print("SEQ real 100x400 prefix", flush=True)
    R, M = synth.gene_expr(100, 400, 5, 0.5, seed=3)
    o = oracle.fit(R, M, 5, 5, seed=3, prec="f32", init_mode=1, row_limit=3, selection=3)
    g = S.stmf_fit(_t(R), _t(M), 5, 5, seed=3, init_mode=1, max_row_visits=3, log_cap=16,
                   selection=3)
    assert _log_rows(g.log) == _log_rows(o.log)
    np.testing.assert_allclose(g.log["e"], o.log["e"], rtol=1e-9)


def test_selection_batched_equals_plain(S):
    # the batched launch runs the same selection per fit
    print("selection batched", flush=True)
    probs = synth.batched_problems(4, seed=70, integer=True, m_range=(12, 80), n_range=(12, 120),
                                   r_range=(2, 4), miss_range=(0.2, 0.5))
    dev = [dict(R=_t(p.R), M=_t(p.M), rank=p.rank, iters=2, seed=900 + p.pid) for p in probs]
    for sel in (1, 2, 3):
        outs, statuses, _ = S.stmf_fit_batched(dev, restarts=1, selection=sel, perm_mode=1)
        assert statuses == [0] * len(probs)
        for p, d, (U, V, T) in zip(probs, dev, outs):
            o = oracle.fit(p.R, p.M, p.rank, 2, seed=d["seed"], prec="f32", selection=sel,
                           perm_mode=1)
            np.testing.assert_array_equal(U[0].cpu().numpy(), o.U)
            np.testing.assert_array_equal(V[0].cpu().numpy(), o.V)
            np.testing.assert_array_equal(T[0].cpu().numpy(), o.traj)


def test_selection_bad_options(S):
    print("selection options", flush=True)
    R, M = synth.int_planted(10, 12, 2, 0.2, seed=14)
    for kw in (dict(selection=4), dict(selection=-1), dict(perm_mode=4), dict(strategy=3)):
        with pytest.raises(S.StmfError):
            S.stmf_fit(_t(R), _t(M), 2, 1, **kw)


# ------------------------------------------------------------------ ByElement
ELEM_CASES = [  # m, n, rank, iters, seed, missing, perm_mode
    (40, 70, 3, 3, 21, 0.3, 3), (70, 150, 4, 2, 22, 0.4, 3), (150, 70, 2, 2, 23, 0.3, 3),
    (1, 40, 2, 2, 24, 0.2, 2), (33, 65, 1, 2, 25, 0.0, 2),
]


@pytest.mark.parametrize("m,n,rank,iters,seed,miss,pm", ELEM_CASES)
@pytest.mark.parametrize("group", [0, 1])
def test_byelement_integer(S, m, n, rank, iters, seed, miss, pm, group):
    print(f"ByElement int {m}x{n} r={rank} perm_mode={pm} group={group}", flush=True)
    R, M = synth.int_planted(m, n, rank, miss, seed=seed, hi=30)
    cap = int(M.sum()) * iters + min(m, n) * iters + 1
    o = oracle.fit(R, M, rank, iters, seed=seed, prec="f32", init_hi=30, strategy=1,
                   perm_mode=pm, log_cap=cap)
    assert o.status == 0
    g = S.stmf_fit(_t(R), _t(M), rank, iters, seed=seed, init_hi=30.0, group_size=group,
                   strategy=1, perm_mode=pm, log_cap=cap)
    _compare(g, o)


def test_byelement_exact_entries_are_skipped(S):
    # every entry exact from the start: no trial at all, as in the oracle
    print("ByElement exact start", flush=True)
    rng = np.random.default_rng(3)
    Us = rng.integers(0, 20, (30, 3)).astype(np.float32)
    Vs = rng.integers(0, 20, (3, 50)).astype(np.float32)
    R = np.max(Us[:, :, None] + Vs[None, :, :], axis=1).astype(np.float32)
    M = np.ones_like(R, np.uint8)
    g = S.stmf_fit(_t(R), _t(M), 3, 3, U0=Us, perm_mode=2, strategy=1, log_cap=200)
    assert g.info["trials"] == 0 and g.info["accepted"] == 0
    np.testing.assert_array_equal(g.traj, [0.0] * 4)


def test_byelement_real(S):
    print("ByElement real 60x150", flush=True)
    R, M = synth.gene_expr(60, 150, 4, 0.5, seed=2)
    cap = int(M.sum()) * 3 + 200
    o = oracle.fit(R, M, 4, 3, seed=2, prec="f32", init_mode=1, strategy=1, perm_mode=3,
                   log_cap=cap)
    g = S.stmf_fit(_t(R), _t(M), 4, 3, seed=2, init_mode=1, strategy=1, perm_mode=3, log_cap=cap)
    _compare(g, o, exact=False)


def test_byelement_gene_expression_prefix(S):
    # the full gene-expression-shaped workload in the cooperative launch:
    # the first row visit (about 1000 entries), record by record
    print("ByElement real 500x2000 prefix", flush=True)
    R, M = synth.gene_expr()
    o = oracle.fit(R, M, 5, 50, seed=2, prec="f32", init_mode=1, row_limit=1, strategy=1,
                   perm_mode=3, log_cap=4000)
    g = S.stmf_fit(_t(R), _t(M), 5, 50, seed=2, init_mode=1, max_row_visits=1, log_cap=4000,
                   strategy=1, perm_mode=3)
    assert len(o.log) > 2
    assert _log_rows(g.log) == _log_rows(o.log)
    np.testing.assert_allclose(g.log["e"], o.log["e"], rtol=1e-9)


def test_byelement_batched_equals_oracle(S):
    print("ByElement batched", flush=True)
    probs = synth.batched_problems(4, seed=71, integer=True, m_range=(12, 80), n_range=(12, 120),
                                   r_range=(2, 4), miss_range=(0.2, 0.5))
    dev = [dict(R=_t(p.R), M=_t(p.M), rank=p.rank, iters=2, seed=950 + p.pid) for p in probs]
    outs, statuses, _ = S.stmf_fit_batched(dev, restarts=1, strategy=1, perm_mode=3)
    assert statuses == [0] * len(probs)
    for p, d, (U, V, T) in zip(probs, dev, outs):
        o = oracle.fit(p.R, p.M, p.rank, 2, seed=d["seed"], prec="f32", strategy=1, perm_mode=3,
                       log_cap=1)
        np.testing.assert_array_equal(U[0].cpu().numpy(), o.U)
        np.testing.assert_array_equal(V[0].cpu().numpy(), o.V)
        np.testing.assert_array_equal(T[0].cpu().numpy(), o.traj)


# ------------------------------------------------------------------ ByMatrix
MAT_CASES = [  # m, n, rank, iters, seed, missing
    (20, 30, 3, 12, 31, 0.3), (40, 70, 3, 15, 32, 0.3), (70, 150, 4, 10, 33, 0.4),
    (150, 70, 2, 10, 34, 0.3), (1, 40, 2, 5, 35, 0.2),
]


@pytest.mark.parametrize("m,n,rank,iters,seed,miss", MAT_CASES)
@pytest.mark.parametrize("group", [0, 1])
def test_bymatrix_integer(S, m, n, rank, iters, seed, miss, group):
    print(f"ByMatrix int {m}x{n} r={rank} it={iters} group={group}", flush=True)
    R, M = synth.int_planted(m, n, rank, miss, seed=seed, hi=30)
    o = oracle.fit(R, M, rank, iters, seed=seed, prec="f32", init_hi=30, strategy=2, perm_mode=2,
                   log_cap=iters + 1)
    assert o.status == 0
    g = S.stmf_fit(_t(R), _t(M), rank, iters, seed=seed, init_hi=30.0, group_size=group,
                   strategy=2, perm_mode=2, log_cap=iters + 1)
    _compare(g, o)


@pytest.mark.parametrize("batch_max", [4, 16])
def test_bymatrix_rounds_of_candidates(S, batch_max):
    # rounds of at most batch_max candidates: the selection's cursor carries
    # across rounds, ties of integer keys included
    print(f"ByMatrix rounds batch_max={batch_max}", flush=True)
    R, M = synth.int_planted(24, 40, 3, 0.3, seed=36, hi=12)
    o = oracle.fit(R, M, 3, 20, seed=36, prec="f32", init_hi=12, strategy=2, perm_mode=2,
                   log_cap=32)
    g = S.stmf_fit(_t(R), _t(M), 3, 20, seed=36, init_hi=12.0, strategy=2, perm_mode=2,
                   batch_max=batch_max, batch_first=batch_max, log_cap=32)
    _compare(g, o)


@pytest.mark.parametrize("batch_max", [64, 512])
def test_bymatrix_exact_start_tries_every_cell(S, batch_max):
    # with 512: batches of both operations span several 128-trial chunks,
    # each trial of a chunk on a row of its own
    print(f"ByMatrix exact start batch_max={batch_max}", flush=True)
    rng = np.random.default_rng(6)
    Us = rng.integers(0, 20, (30, 2)).astype(np.float32)
    Vs = rng.integers(0, 20, (2, 50)).astype(np.float32)
    R = np.max(Us[:, :, None] + Vs[None, :, :], axis=1).astype(np.float32)
    M = np.ones_like(R, np.uint8)
    o = oracle.fit(R, M, 2, 3, prec="f32", init_mode=2, U0=Us, perm_mode=2, strategy=2, seed=6)
    g = S.stmf_fit(_t(R), _t(M), 2, 3, seed=6, U0=Us, perm_mode=2, strategy=2, log_cap=8,
                   batch_max=batch_max, batch_first=batch_max)
    assert g.info["accepted"] == 0 and g.info["trials"] + g.info["noops"] == 1500
    assert g.info["trials"] == o.stats["trials"] and g.info["noops"] == o.stats["noops"]
    np.testing.assert_array_equal(g.traj, [0.0] * 4)


def test_bymatrix_real(S):
    print("ByMatrix real 60x150", flush=True)
    R, M = synth.gene_expr(60, 150, 4, 0.5, seed=2)
    o = oracle.fit(R, M, 4, 12, seed=2, prec="f32", init_mode=1, strategy=2, perm_mode=2,
                   log_cap=16)
    g = S.stmf_fit(_t(R), _t(M), 4, 12, seed=2, init_mode=1, strategy=2, perm_mode=2, log_cap=16)
    _compare(g, o, exact=False)


def test_bymatrix_gene_expression_prefix(S):
    # the full gene-expression-shaped workload in the cooperative launch: the
    # first 3 iterations (each keys and orders 500,000 cells), record by record
    print("ByMatrix real 500x2000 prefix", flush=True)
    R, M = synth.gene_expr()
    o = oracle.fit(R, M, 5, 50, seed=2, prec="f32", init_mode=1, row_limit=3, strategy=2,
                   perm_mode=2, log_cap=8)
    g = S.stmf_fit(_t(R), _t(M), 5, 50, seed=2, init_mode=1, max_row_visits=3, log_cap=8,
                   strategy=2, perm_mode=2)
    assert _log_rows(g.log) == _log_rows(o.log)
    np.testing.assert_allclose(g.log["e"], o.log["e"], rtol=1e-9)


def test_bymatrix_not_batched(S):
    print("ByMatrix batched refused", flush=True)
    probs = synth.batched_problems(1, seed=72, integer=True, m_range=(12, 20), n_range=(12, 20),
                                   r_range=(2, 2), miss_range=(0.2, 0.3))
    dev = [dict(R=_t(p.R), M=_t(p.M), rank=p.rank, iters=2, seed=1) for p in probs]
    with pytest.raises(S.StmfError):
        S.stmf_fit_batched(dev, restarts=1, strategy=2)


# ------------------------------------------------------------------ maximum rank
@pytest.mark.parametrize("strategy,sel,pm,iters", [
    (0, 0, 0, 3), (0, 1, 0, 3), (0, 2, 0, 3), (0, 3, 0, 1), (1, 0, 3, 2), (2, 0, 2, 12),
])
def test_every_strategy_at_rank_64(S, strategy, sel, pm, iters):
    # rank 64 (the largest supported): eight blocks of eight staged
    # components, sixteen per candidate thread in the batch list
    print(f"rank 64 strategy={strategy} selection={sel}", flush=True)
    R, M = synth.int_planted(20, 30, 64, 0.25, seed=40 + strategy * 4 + sel, hi=40)
    cap = int(M.sum()) * iters + 64
    o = oracle.fit(R, M, 64, iters, seed=5, prec="f32", init_hi=40, strategy=strategy,
                   selection=sel, perm_mode=pm, log_cap=cap)
    assert o.status == 0
    g = S.stmf_fit(_t(R), _t(M), 64, iters, seed=5, init_hi=40.0, strategy=strategy, selection=sel,
                   perm_mode=pm, log_cap=cap)
    _compare(g, o)
