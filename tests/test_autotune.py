"""Autotuner: the search loop, batch signatures and the cache (CPU), and a
measured search on the GPU whose every trial must reproduce the statistics."""
import json

import numpy as np
import pytest

import paper_2509_03653_amd as nsgc
from paper_2509_03653_amd import autotune as at


def test_size_classes_match_the_planner_classing():
    off = np.array([0, 0, 1, 3, 4, 1028, 1028 + (1 << 20)], np.int64)
    pc = at.size_classes(off)
    assert pc.shape == (33,)
    # sizes 0,1,2,1,1024,2^20 -> classes 0,0,1,0,10,20
    assert pc[0] == 2 and pc[1] == 2 and pc[10] == 1024 and pc[20] == 1 << 20
    assert pc.sum() == off[-1]


def test_signature_is_coarse_and_stable():
    a = np.concatenate([[0], np.cumsum(np.full(64, 1 << 17))]).astype(np.int64)
    b = a.copy()
    b[1:] += 5                    # a few packets more in the first window only
    assert at.signature(a) == at.signature(b)
    c = np.concatenate([[0], np.cumsum(np.full(64, 1 << 12))]).astype(np.int64)
    assert at.signature(a) != at.signature(c)
    assert at.signature(np.array([0], np.int64)) == at.signature(np.array([7], np.int64))


def test_apply_point_scales_only_present_classes():
    base = nsgc.default_tune().to_dict()
    d = at.apply_point(base, {"blocks_per_cu": 3, "link_scale": 2.0, "rc_scale": 0.5,
                              "wave_target": 0}, [17])
    assert d["blocks_per_cu"] == 3
    assert d["cls"][17][0] == 2 * base["cls"][17][0]
    assert d["cls"][17][1] == base["cls"][17][1] // 2
    assert d["cls"][17][2] == base["cls"][17][2] // 2
    # row_scale multiplies the row target on top of rc_scale, in any key order
    for pt in ({"row_scale": 2.0, "rc_scale": 0.5}, {"rc_scale": 0.5, "row_scale": 2.0}):
        e = at.apply_point(base, pt, [17])
        assert e["cls"][17][1] == base["cls"][17][1]
        assert e["cls"][17][2] == base["cls"][17][2] // 2
    assert d["cls"][17][3] == 0 and base["cls"][17][3] > 0
    assert d["cls"][16] == base["cls"][16]
    nsgc.Tune.from_dict(d)   # a valid tuning structure


def test_every_point_of_the_space_is_a_valid_tuning():
    base = nsgc.default_tune().to_dict()
    before = nsgc.get_tune().to_dict()
    try:
        for knob, values in at.SPACE:
            for v in values:
                d = at.apply_point(base, {knob: v}, range(33))
                nsgc.set_tune(nsgc.Tune.from_dict(d))   # raises if invalid
    finally:
        nsgc.set_tune(nsgc.Tune.from_dict(before))


def test_search_finds_the_separable_optimum():
    # cost model with a known optimum; coordinate descent must reach it
    opt = {"blocks_per_cu": 3, "link_slots_log2": 11, "rc_slots_log2": 13, "tile_log2": 14,
           "small_max": 512, "link_scale": 2.0, "max_link_buckets_log2": 11, "rc_scale": 0.5,
           "row_scale": 2.0, "wave_target": 128, "combine_probes": 64}
    assert set(opt) == {k for k, _ in at.SPACE}
    calls = []

    rank = {k: {v: i for i, v in enumerate(vals)} for k, vals in at.SPACE}

    def measure(p):
        calls.append(dict(p))
        return 1.0 + sum(abs(rank[k][p[k]] - rank[k][v]) for k, v in opt.items())

    start = at.start_point(nsgc.default_tune().to_dict())
    res = at.search(measure, start)
    assert res.point == opt
    assert res.ms == pytest.approx(1.0)
    assert res.start_ms > res.ms
    assert len(res.trials) == len(calls)
    assert len(calls) <= 1 + sum(len(v) for _, v in at.SPACE)


def test_search_keeps_incumbent_within_margin_and_respects_limits():
    start = at.start_point(nsgc.default_tune().to_dict())
    res = at.search(lambda p: 1.0 - 0.001 * p["blocks_per_cu"], start, margin=0.02)
    assert res.point == start                   # 0.1% gains are below the margin
    res = at.search(lambda p: 1.0, start, max_trials=3)
    assert len(res.trials) == 3

    t = [0.0]

    def clock():
        t[0] += 10.0
        return t[0]

    res = at.search(lambda p: 1.0, start, budget_s=25.0, clock=clock)
    assert len(res.trials) <= 3


def test_search_propagates_measure_errors():
    def bad(p):
        if p["blocks_per_cu"] == 1:
            raise at.MismatchError("different statistics")
        return 1.0

    with pytest.raises(at.MismatchError):
        at.search(bad, at.start_point(nsgc.default_tune().to_dict()))


def test_cache_roundtrip_and_versioning(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert at.cache_load(p) == {}
    at.cache_store(p, "k1", {"tune": {"small_max": 7}, "ms": 1.5})
    at.cache_store(p, "k2", {"tune": {"small_max": 9}, "ms": 2.5})
    got = at.cache_load(p)
    assert got["k1"]["ms"] == 1.5 and got["k2"]["tune"]["small_max"] == 9
    with open(p) as f:
        data = json.load(f)
    data["version"] = -1
    with open(p, "w") as f:
        json.dump(data, f)
    assert at.cache_load(p) == {}
    with open(p, "w") as f:
        f.write("{not json")
    assert at.cache_load(p) == {}


@pytest.mark.gpu
def test_measured_search_is_exact_and_cached(tmp_path):
    import torch

    import oracle
    import synth
    from gpu_util import assert_same, say, to_gpu

    wl = synth.uneven_batch(seed=3, num_windows=24, lo_log2=8, hi_log2=17)
    src, dst = wl.generate()
    want = oracle.window_stats(src, dst, wl.offsets, threads=8)
    s, d = to_gpu(src), to_gpu(dst)
    path = str(tmp_path / "tune.json")
    space = (("blocks_per_cu", (1, 2)), ("link_slots_log2", (11, 12)), ("small_max", (512, 1024)))
    before = nsgc.get_tune()
    try:
        say("[gpu] autotune search")
        r = at.tune_for(s, d, wl.offsets, cache_path=path, space=space, repeats=2, warmup=1,
                        budget_s=60)
        assert not r["cached"] and r["ms"] > 0 and r["trials"] >= 2
        assert nsgc.get_tune().to_dict() == r["tune"]
        out = nsgc.window_stats(s, d, wl.offsets)
        torch.cuda.synchronize()
        assert_same(out.cpu().numpy().view(np.uint64), want, "autotuned")
        say("[gpu] autotune cache hit")
        r2 = at.tune_for(s, d, wl.offsets, cache_path=path, space=space)
        assert r2["cached"] and r2["tune"] == r["tune"]
        assert at.cached(wl.offsets, cache_path=path).to_dict() == r["tune"]
    finally:
        nsgc.set_tune(before)
