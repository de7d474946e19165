"""GPU tests of serving: the continuous-batching engine (admit / tick / poll /
retire) and the serving loop over it.  A job's arithmetic never depends on
which other jobs share its launches or when it was admitted: each result
equals stmf_fit alone with the job's group size (one workgroup by default;
the smaller of the engine's group size and the job's tile count otherwise)
and the same seed, bit for bit, on real-valued data."""
import numpy as np
import pytest

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


def _jobs(seed, count):
    probs = synth.batched_problems(count, seed=seed, integer=False, m_range=(16, 90),
                                   n_range=(16, 140), r_range=(2, 4), miss_range=(0.2, 0.6))
    return [dict(R=_t(p.R), M=_t(p.M), rank=p.rank, iters=3, seed=700 + p.pid) for p in probs]


def _alone(S, j, G=1):
    return S.stmf_fit(j["R"], j["M"], j["rank"], j["iters"], seed=j["seed"], group_size=G)


def _group(gcap, m, n):
    # a job's workgroups: the engine's group size (0: no limit), at most the
    # job's 64 x 64 tiles of the working (wide) orientation (the device holds
    # more workgroups at once than these jobs have tiles)
    mw, nw = min(m, n), max(m, n)
    tiles = -(-mw // 64) * -(-nw // 64)
    return tiles if gcap == 0 else max(1, min(gcap, tiles))


def _plain(S, j):
    # stmf_fit with its own choice of group: what an engine with group size 0
    # reproduces
    return S.stmf_fit(j["R"], j["M"], j["rank"], j["iters"], seed=j["seed"])


def _same(res, ref):
    np.testing.assert_array_equal(res.U.cpu().numpy(), ref.U.cpu().numpy())
    np.testing.assert_array_equal(res.V.cpu().numpy(), ref.V.cpu().numpy())
    np.testing.assert_array_equal(res.traj, ref.traj)


def _drain(S, eng, slots, rows, limit=10000):
    out = {}
    for _ in range(limit):
        if len(out) == len(slots):
            return out
        S.stmf_batch_tick(eng, rows)
        for s in slots:
            if s not in out and S.stmf_engine_poll(eng, s):
                out[s] = S.stmf_engine_retire(eng, s)
    raise AssertionError("jobs did not finish")


@pytest.mark.parametrize("gcap", [1, 0])
def test_engine_results_equal_plain(S, gcap):
    print(f"engine vs plain group {gcap}", flush=True)
    jobs = _jobs(60, 4)
    eng = S.stmf_engine_create(256 << 20, 8, group_size=gcap)
    try:
        slots = [S.stmf_engine_admit(eng, j["R"], j["M"], j["rank"], j["iters"], j["seed"]) for j in jobs]
        assert None not in slots and len(set(slots)) == len(slots)
        res = _drain(S, eng, slots, rows=5)
    finally:
        S.stmf_engine_destroy(eng)
    for j, s in zip(jobs, slots):
        G = _group(gcap, *j["R"].shape)
        assert res[s].info["group_size"] == G
        _same(res[s], _alone(S, j, G))
        if gcap == 0:
            _same(res[s], _plain(S, j))


def test_engine_alone_vs_mix(S):
    print("engine alone vs mix", flush=True)
    jobs = _jobs(61, 4)
    x = jobs[0]
    eng = S.stmf_engine_create(256 << 20, 8)
    try:
        sx = S.stmf_engine_admit(eng, x["R"], x["M"], x["rank"], x["iters"], x["seed"])
        alone = _drain(S, eng, [sx], rows=3)[sx]
        # the same job admitted into a running mix, after two ticks of the others
        others = [S.stmf_engine_admit(eng, j["R"], j["M"], j["rank"], j["iters"], j["seed"])
                  for j in jobs[1:]]
        S.stmf_batch_tick(eng, 2)
        S.stmf_batch_tick(eng, 2)
        sx2 = S.stmf_engine_admit(eng, x["R"], x["M"], x["rank"], x["iters"], x["seed"])
        mix = _drain(S, eng, others + [sx2], rows=3)
    finally:
        S.stmf_engine_destroy(eng)
    _same(mix[sx2], alone)
    _same(alone, _plain(S, x))
    for j, s in zip(jobs[1:], others):
        _same(mix[s], _plain(S, j))


def test_engine_admission_by_footprint(S):
    print("engine admission", flush=True)
    j = _jobs(62, 1)[0]
    m, n = j["R"].shape
    fp = S.stmf_job_footprint(m, n, j["rank"], j["iters"])
    assert fp > 0
    # room for one job, not two (one workgroup per job: the footprint of
    # stmf_job_footprint)
    eng = S.stmf_engine_create(65536 + fp + fp // 2, 4, group_size=1)
    try:
        assert S.stmf_engine_job_footprint(eng, m, n, j["rank"], j["iters"]) == fp
        s1 = S.stmf_engine_admit(eng, j["R"], j["M"], j["rank"], j["iters"], j["seed"])
        assert s1 is not None
        assert S.stmf_engine_admit(eng, j["R"], j["M"], j["rank"], j["iters"], j["seed"]) is None
        r1 = _drain(S, eng, [s1], rows=4)[s1]
        s2 = S.stmf_engine_admit(eng, j["R"], j["M"], j["rank"], j["iters"], j["seed"])
        assert s2 is not None
        r2 = _drain(S, eng, [s2], rows=4)[s2]
    finally:
        S.stmf_engine_destroy(eng)
    _same(r1, r2)


def test_engine_slot_limit(S):
    print("engine slots", flush=True)
    jobs = _jobs(63, 3)
    eng = S.stmf_engine_create(256 << 20, 2)
    try:
        a = S.stmf_engine_admit(eng, jobs[0]["R"], jobs[0]["M"], jobs[0]["rank"], 2, 1)
        b = S.stmf_engine_admit(eng, jobs[1]["R"], jobs[1]["M"], jobs[1]["rank"], 2, 2)
        assert a is not None and b is not None
        assert S.stmf_engine_admit(eng, jobs[2]["R"], jobs[2]["M"], jobs[2]["rank"], 2, 3) is None
        _drain(S, eng, [a, b], rows=50)
    finally:
        S.stmf_engine_destroy(eng)


def test_serve_loop_results_match_alone(S):
    print("serve loop", flush=True)
    from paper_2205_06619_amd import serve
    jobs = serve.synthetic_jobs(8, rate_per_s=200.0, seed=64, m_range=(16, 80), n_range=(16, 120),
                                r_range=(2, 4), miss_range=(0.2, 0.6), iters=3)
    backend = serve.EngineBackend(256 << 20, 8)
    try:
        st = serve.Server(backend, rows_per_tick=4).run(jobs)
    finally:
        backend.close()
    assert st.jobs == 8 and 0 < st.p50_ms <= st.p99_ms
    assert st.max_resident >= 1 and st.ticks >= 1
    for j in jobs:
        assert j.finished >= j.arrival
        ref = S.stmf_fit(j.R, j.M, j.rank, j.iters, seed=j.seed)
        _same(j.result, ref)


@pytest.mark.parametrize("gcap", [1, 4, 0])
def test_engine_graph_ticks_equal_eager_ticks(S, gcap):
    # the same stream of admissions and ticks through an engine whose ticks
    # replay a captured graph and one that launches eagerly: every job's
    # result is identical (the graph is replayed many times, re-captured as
    # the resident set changes, with host polls between the replays)
    print(f"engine graph vs eager group {gcap}", flush=True)
    jobs = _jobs(65, 5) if gcap == 1 else _wide_jobs(65, 5)
    engs = [S.stmf_engine_create(256 << 20, 8, group_size=gcap),
            S.stmf_engine_create(256 << 20, 8, group_size=gcap)]
    S.stmf_engine_set_graph(engs[1], False)
    try:
        slots = [[], []]
        results = [{}, {}]
        for e, eng in enumerate(engs):
            for j in jobs[:2]:
                slots[e].append(S.stmf_engine_admit(eng, j["R"], j["M"], j["rank"], j["iters"], j["seed"]))
        for step in range(400):
            if step == 3:
                for e, eng in enumerate(engs):
                    for j in jobs[2:]:
                        slots[e].append(S.stmf_engine_admit(eng, j["R"], j["M"], j["rank"], j["iters"],
                                                            j["seed"]))
            for e, eng in enumerate(engs):
                S.stmf_batch_tick(eng, 2)
                for s in slots[e]:
                    if s not in results[e] and S.stmf_engine_poll(eng, s):
                        results[e][s] = S.stmf_engine_retire(eng, s)
            if all(len(results[e]) == len(jobs) for e in range(2)):
                break
        assert all(len(results[e]) == len(jobs) for e in range(2))
    finally:
        for eng in engs:
            S.stmf_engine_destroy(eng)
    for q, j in enumerate(jobs):
        a, b = results[0][slots[0][q]], results[1][slots[1][q]]
        _same(a, b)
        G = _group(gcap, *j["R"].shape)
        assert a.info["group_size"] == G
        _same(a, _alone(S, j, G))


def _wide_jobs(seed, count):
    # shapes of 1 to 12 tiles, so groups of 1 to 4 workgroups meet in a launch
    probs = synth.batched_problems(count, seed=seed, integer=False, m_range=(40, 200),
                                   n_range=(60, 260), r_range=(2, 4), miss_range=(0.2, 0.6))
    return [dict(R=_t(p.R), M=_t(p.M), rank=p.rank, iters=2, seed=800 + p.pid) for p in probs]


@pytest.mark.parametrize("gcap", [4, 16])
def test_engine_groups_equal_plain_with_that_group(S, gcap):
    print(f"engine groups {gcap}", flush=True)
    jobs = _wide_jobs(66 + gcap, 6)
    eng = S.stmf_engine_create(512 << 20, 8, group_size=gcap)
    try:
        for j in jobs:
            m, n = j["R"].shape
            assert S.stmf_engine_job_footprint(eng, m, n, j["rank"], j["iters"]) >= \
                S.stmf_job_footprint(m, n, j["rank"], j["iters"])
        slots = [S.stmf_engine_admit(eng, j["R"], j["M"], j["rank"], j["iters"], j["seed"]) for j in jobs]
        assert None not in slots
        res = _drain(S, eng, slots, rows=7)
    finally:
        S.stmf_engine_destroy(eng)
    Gs = [_group(gcap, *j["R"].shape) for j in jobs]
    assert max(Gs) > 1
    for j, s, G in zip(jobs, slots, Gs):
        assert res[s].info["group_size"] == G
        _same(res[s], _alone(S, j, G))


def test_engine_groups_over_several_launches(S):
    # two jobs of 5 x 65 tiles with groups as large as the device holds at
    # once: the pair does not fit in one launch, so a tick runs two
    print("engine groups over launches", flush=True)
    rng = np.random.default_rng(67)
    jobs = []
    for q in range(2):
        R = rng.random((300, 4100)).astype(np.float32)
        M = (rng.random((300, 4100)) < 0.5).astype(np.uint8)
        M[:, 0] = 1
        M[0, :] = 1
        jobs.append(dict(R=_t(R), M=_t(M), rank=3, iters=1, seed=900 + q))
    eng = S.stmf_engine_create(1 << 30, 4, group_size=1024)
    try:
        slots = [S.stmf_engine_admit(eng, j["R"], j["M"], j["rank"], j["iters"], j["seed"]) for j in jobs]
        assert None not in slots
        res = _drain(S, eng, slots, rows=100)
    finally:
        S.stmf_engine_destroy(eng)
    for j, s in zip(jobs, slots):
        G = res[s].info["group_size"]
        assert 64 <= G <= 325
        ref = _alone(S, j, G)
        assert ref.info["group_size"] == G
        _same(res[s], ref)


@pytest.mark.parametrize("gcap", [1, 0])
def test_engine_zero_passes_and_tiny_jobs(S, gcap):
    print(f"engine edge jobs group={gcap}", flush=True)
    jobs = _wide_jobs(68, 2)
    jobs[0]["iters"] = 0
    for shape, seed in (((1, 70), 55), ((90, 1), 56)):
        R, M = synth.int_planted(shape[0], shape[1], 1, 0.0, seed=seed)
        jobs.append(dict(R=_t(R), M=_t(M), rank=1, iters=2, seed=seed))
    eng = S.stmf_engine_create(256 << 20, 8, group_size=gcap)
    try:
        slots = [S.stmf_engine_admit(eng, j["R"], j["M"], j["rank"], j["iters"], j["seed"]) for j in jobs]
        assert None not in slots
        res = _drain(S, eng, slots, rows=3)
    finally:
        S.stmf_engine_destroy(eng)
    for j, s in zip(jobs, slots):
        _same(res[s], _alone(S, j, _group(gcap, *j["R"].shape)))
