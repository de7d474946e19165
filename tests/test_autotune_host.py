"""Host logic of the launch-shape autotuner: buckets, the choice rule and
the JSON cache (no GPU)."""
import json

from paper_2205_06619_amd import autotune


def test_bucket_rounds_the_working_shape_up():
    assert autotune.bucket(200, 100, 3) == "128x256r4"
    assert autotune.bucket(100, 200, 3) == "128x256r4"
    assert autotune.bucket(500, 2000, 5) == "512x2048r8"
    assert autotune.bucket(1, 1, 1) == "1x1r1"


def test_choose_takes_the_fastest_and_the_first_on_ties():
    t = {(0, 0): 5.0, (16, 0): 3.0, (64, 0): 3.0, (0, 256): 4.0}
    best, times = autotune.choose(list(t), lambda bf, bm: t[(bf, bm)])
    assert best == (16, 0)
    assert times == {"0,0": 5.0, "16,0": 3.0, "64,0": 3.0, "0,256": 4.0}


def test_choose_keeps_the_best_of_repeats():
    seq = iter([9.0, 2.0, 4.0, 3.0])
    best, times = autotune.choose([(0, 0), (16, 0)], lambda bf, bm: next(seq), repeats=2)
    assert best == (0, 0) and times["0,0"] == 2.0 and times["16,0"] == 3.0


def test_cache_round_trip(tmp_path):
    path = tmp_path / "sub" / "tune.json"
    c = autotune.Cache(str(path))
    assert c.get("fit:8x8r2") is None
    c.put("fit:8x8r2", {"batch_first": 16, "batch_max": 256, "times_ms": {"16,256": 1.0}})
    again = autotune.Cache(str(path))
    assert again.get("fit:8x8r2")["batch_max"] == 256
    assert json.loads(path.read_text())["fit:8x8r2"]["batch_first"] == 16


def test_candidates_are_valid_options():
    for bf, bm in autotune.CANDIDATES:
        assert 0 <= bf and 0 <= bm <= 1024
        assert bm == 0 or bf <= bm


class _Info:
    def __init__(self, ms):
        self.info = {"kernel_ms": ms}


class _Shape:
    shape = (300, 4000)


def test_tune_fit_prefix_and_cache(tmp_path, monkeypatch):
    # the fit itself is replaced by a timer of the candidate; what is checked
    # is the prefix each candidate runs, the choice and the cache entry
    from paper_2205_06619_amd import stmf
    seen = []

    def fake_fit(R, M, rank, passes, seed=0, batch_first=0, batch_max=0, max_row_visits=0, **kw):
        seen.append((batch_first, batch_max, max_row_visits))
        return _Info(10.0 - (batch_first == 64 and batch_max == 0))

    monkeypatch.setattr(stmf, "stmf_fit", fake_fit)
    cache = autotune.Cache(str(tmp_path / "t.json"))
    got = autotune.tune_fit(_Shape(), None, 20, visits=40, cache=cache)
    assert got == {"batch_first": 64, "batch_max": 0}
    assert [v for _, _, v in seen] == [40] * len(autotune.CANDIDATES)
    assert cache.get("fit:512x4096r32")["batch_first"] == 64
    seen.clear()
    assert autotune.tune_fit(_Shape(), None, 20, cache=cache) == got and not seen
    autotune.tune_fit(_Shape(), None, 20, passes=2)
    assert {v for _, _, v in seen} == {600}


def test_sample_spreads_over_the_sizes():
    class P:
        def __init__(self, n):
            self.n = n

        def numel(self):
            return self.n

    probs = [dict(R=P(n), pid=n) for n in (5, 50, 20, 80, 10, 40, 70, 30)]
    got = [p["pid"] for p in autotune.sample_problems(probs, 3)]
    assert got == [80, 30, 5]           # largest, middle, smallest
    assert len(autotune.sample_problems(probs, 20)) == 8
    assert all(g in (1, 2, 4, 8, 16) for g in autotune.GROUP_SIZES)
