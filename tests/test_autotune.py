"""Autotuner selection and persistence (CPU only: the measurement is injected)."""
import numpy as np

from paper_1704_05132_amd import autotune
from paper_1704_05132_amd.instances import draw_instance


def test_pick_returns_fastest_and_all_timings():
    times = {2: 5.0, 4: 3.0, 8: 3.0}
    best, timings = autotune.pick([dict(waves=w) for w in (2, 4, 8)], lambda c: times[c["waves"]])
    assert best == {"waves": 4}               # ties keep the earlier candidate
    assert [ms for _, ms in timings] == [5.0, 3.0, 3.0]


def test_signature_distinguishes_workloads():
    rng = np.random.default_rng(1)
    a = [draw_instance(rng, 10, 12), draw_instance(rng, 30, 52)]
    b = [draw_instance(rng, 10, 12), draw_instance(rng, 30, 24)]
    assert autotune.signature(a, 8) == "n2_K10-30_T12-52_c8"
    assert autotune.signature(a, 8) != autotune.signature(b, 8)
    assert autotune.signature(a, 8) != autotune.signature(a, 16)


def test_table_round_trip(tmp_path):
    t = autotune.TuneTable(tmp_path / "tune.json")
    assert t.get("k") is None
    t.put("k", {"waves": 4, "lds": 0}, [({"waves": 4, "lds": 0}, 1.5)])
    t2 = autotune.TuneTable(tmp_path / "tune.json")
    assert t2.get("k")["choice"] == {"waves": 4, "lds": 0}
    assert t2.get("k")["timings_ms"] == [[{"waves": 4, "lds": 0}, 1.5]]


def test_search_options_map_every_key():
    from paper_1704_05132_amd import vns
    assert autotune.search_options(dict(waves=4, lds=0, spec=0)) == {vns.OPT_RUN_WAVES: 4, vns.OPT_RUN_LDS: 0,
                                                                      vns.OPT_SPECULATE: 0}
    assert autotune.search_options(dict(spec=1, spec_waves=9, lds=65536)) == {vns.OPT_SPECULATE: 1,
                                                                               vns.OPT_SPEC_WAVES: 9,
                                                                               vns.OPT_RUN_LDS: 65536}
    assert autotune.search_options({"group": 8}) == {}
    assert autotune.search_options(dict(waves=2, state=1)) == {vns.OPT_RUN_WAVES: 2, vns.OPT_STATE_LDS: 1}
    assert autotune.search_options(dict(waves=4, iters=6)) == {vns.OPT_RUN_WAVES: 4, vns.OPT_SPEC_ITERS: 6}


def test_eval_options_map_group_and_spread():
    from paper_1704_05132_amd import vns
    assert autotune.eval_options({"group": 5}) == {vns.OPT_EVAL_SPREAD: 0, vns.OPT_EVAL_GROUP: 5}
    assert autotune.eval_options({"spread": 8}) == {vns.OPT_EVAL_SPREAD: 8}
    assert autotune.eval_options(dict(waves=4, iters=12)) == {vns.OPT_EVAL_SPREAD: 0}
    assert {c.get("spread") for c in autotune.EVAL_CANDIDATES} >= {4, 8, 12, 16}


def test_candidates_cover_both_search_kernels():
    kinds = {c.get("spec", 0) for c in autotune.SEARCH_CANDIDATES}
    assert kinds == {0, 1}
    for c in autotune.SEARCH_CANDIDATES:
        if c.get("spec"):
            assert c["spec_waves"] % 3 == 0 and 3 <= c["spec_waves"] <= 16   # whole groups of three waves
            assert "iters" not in c   # speculative iterations run the one-wavefront-per-product VND
        assert 1 <= c.get("iters", 1) <= 16
    assert any(c.get("iters", 1) > 1 for c in autotune.SEARCH_CANDIDATES)
