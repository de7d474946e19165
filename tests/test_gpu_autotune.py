"""GPU tests of the autotuner: a tuned launch shape changes timing only, so
fits and batched fits with the tuned options equal those with the defaults,
bit for bit."""
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


def test_tuned_fit_equals_default(S, tmp_path):
    print("autotune fit", flush=True)
    from paper_2205_06619_amd import autotune
    R, M = synth.gene_expr(120, 400, 4, 0.5, seed=9)
    Rd, Md = _t(R), _t(M)
    cache = autotune.Cache(str(tmp_path / "t.json"))
    opts = autotune.tune_fit(Rd, Md, 4, passes=1, seed=9, cache=cache, init_mode=1)
    assert (opts["batch_first"], opts["batch_max"]) in autotune.CANDIDATES
    assert cache.get("fit:" + autotune.bucket(120, 400, 4))["batch_max"] == opts["batch_max"]
    a = S.stmf_fit(Rd, Md, 4, 3, seed=9, init_mode=1)
    b = S.stmf_fit(Rd, Md, 4, 3, seed=9, init_mode=1, **opts)
    np.testing.assert_array_equal(a.U.cpu().numpy(), b.U.cpu().numpy())
    np.testing.assert_array_equal(a.V.cpu().numpy(), b.V.cpu().numpy())
    np.testing.assert_array_equal(a.traj, b.traj)
    # a second call reads the cache
    assert autotune.tune_fit(Rd, Md, 4, cache=cache) == opts


def test_tuned_batched_equals_default(S):
    print("autotune batched", flush=True)
    from paper_2205_06619_amd import autotune
    probs = synth.batched_problems(10, seed=80, integer=True, m_range=(20, 120), n_range=(20, 200),
                                   r_range=(2, 6), miss_range=(0.2, 0.6))
    dev = [dict(R=_t(p.R), M=_t(p.M), rank=p.rank, iters=3, seed=500 + p.pid) for p in probs]
    opts = autotune.tune_batched(dev, restarts=2, sample=4, iters=1)
    assert opts["group_size"] in autotune.GROUP_SIZES
    a, sa, _ = S.stmf_fit_batched(dev, restarts=2)
    b, sb, _ = S.stmf_fit_batched(dev, restarts=2, **opts)
    assert sa == sb == [0] * len(probs)
    for (Ua, Va, Ta), (Ub, Vb, Tb) in zip(a, b):
        np.testing.assert_array_equal(Ua.cpu().numpy(), Ub.cpu().numpy())
        np.testing.assert_array_equal(Va.cpu().numpy(), Vb.cpu().numpy())
        np.testing.assert_array_equal(Ta.cpu().numpy(), Tb.cpu().numpy())
