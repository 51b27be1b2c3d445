"""Host-only checks of the C ABI: exports, argument validation, planner.

No device work happens here: invalid arguments are rejected before any HIP
call, and nsgc_plan_inspect is pure host code.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2509_03653_amd as nsgc
from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "nsgc.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nsgc_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert header_functions() == sorted(nsgc.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = nsgc.library()
    for name in header_functions():
        assert hasattr(lib, name), name
    out = subprocess.check_output(["nm", "-D", "--defined-only", nsgc.LIB_PATH]).decode()
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in header_functions():
        assert name in exported, name


def test_noalloc_limits_match_the_header():
    text = open(HEADER).read()
    scratch = re.search(r"#define NSGC_NOALLOC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", text)
    plan = re.search(r"#define NSGC_NOALLOC_PLAN_BYTES \((\d+)ull << (\d+)\)", text)
    assert scratch and plan
    assert int(scratch[1]) << int(scratch[2]) == nsgc.NOALLOC_SCRATCH_BYTES
    assert int(plan[1]) << int(plan[2]) == nsgc.NOALLOC_PLAN_BYTES
    assert nsgc.NOALLOC_PLAN_BYTES % 256 == 0 < nsgc.NOALLOC_PLAN_BYTES < nsgc.NOALLOC_SCRATCH_BYTES


def test_status_strings():
    lib = nsgc.library()
    for code in range(-7, 1):
        assert lib.nsgc_status_string(code)
    assert lib.nsgc_status_string(-99) == b"unknown status"


def _call(fn, src, dst, off, w, out):
    return fn(ctypes.c_void_p(src), ctypes.c_void_p(dst),
              ctypes.c_void_p(off.ctypes.data if off is not None else 0), w,
              ctypes.c_void_p(out), ctypes.c_void_p(0))


@pytest.mark.parametrize("entry", ["nsgc_window_stats", "nsgc_window_stats_plain",
                                   "nsgc_window_stats_noalloc"])
def test_invalid_arguments_rejected_before_any_device_work(entry):
    fn = getattr(nsgc.library(), entry)
    off = np.array([0, 4, 8], np.int64)
    fake = 0x1000   # never dereferenced: validation fails first
    assert _call(fn, fake, fake, off, -1, fake) == -1           # negative count
    assert _call(fn, fake, fake, None, 2, fake) == -1           # no offsets
    assert _call(fn, fake, fake, off, 2, 0) == -1               # no output
    assert _call(fn, fake, fake, off, 2, fake + 4) == -1        # misaligned output
    assert _call(fn, 0, fake, off, 2, fake) == -1               # packets but no src
    assert _call(fn, 0, 0, off, 0, 0) == 0                      # zero windows: no-op
    bad = np.array([0, 4, 3], np.int64)
    assert _call(fn, fake, fake, bad, 2, fake) == -2            # decreasing
    neg = np.array([-1, 4], np.int64)
    assert _call(fn, fake, fake, neg, 1, fake) == -2            # negative
    huge = np.array([0, 1 << 32], np.int64)
    assert _call(fn, fake, fake, huge, 1, fake) == -2           # window of 2^32 packets


def test_tune_roundtrip_and_validation():
    t = nsgc.default_tune()
    d = t.to_dict()
    assert d["small_max"] >= 0 and 11 <= d["tile_log2"] <= 14
    t2 = nsgc.Tune.from_dict(d)
    assert t2.to_dict() == d
    assert d["max_sweeps_log2"] == 24
    for k, v in (("tile_log2", 9), ("tile_log2", 15), ("link_slots_log2", 13),
                 ("rc_slots_log2", 14), ("small_max", 2049), ("blocks_per_cu", 0),
                 ("max_link_buckets_log2", 13), ("max_rc_buckets_log2", 13),
                 ("max_link_buckets_log2", -1), ("max_sweeps_log2", 25), ("max_sweeps_log2", -1),
                 ("combine_probes", -1), ("combine_probes", 65), ("row_complete", 2),
                 ("row_complete", -1)):
        with pytest.raises(nsgc.NsgcError):
            nsgc.set_tune(nsgc.Tune.from_dict(dict(d, **{k: v})))
        assert nsgc.get_tune().to_dict() == d, k
    bad_cls = [list(r) for r in d["cls"]]
    bad_cls[5][1] = 63
    with pytest.raises(nsgc.NsgcError):
        nsgc.set_tune(nsgc.Tune.from_dict(dict(d, cls=bad_cls)))
    assert nsgc.get_tune().to_dict() == d


def test_check_valid_flags_marked_windows():
    ok = np.zeros((3, 9), np.uint64)
    nsgc.check_valid(ok)
    bad = ok.copy()
    bad[1, 0] = np.uint64(1 << 63) | np.uint64(17)
    with pytest.raises(nsgc.NsgcError):
        nsgc.check_valid(bad)


def test_plan_tiers_and_cutover():
    small_max = nsgc.get_tune().small_max
    sizes = [0, 1, small_max, small_max + 1, 1 << 17, 1 << 23]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    p = nsgc.plan_inspect(off)
    assert list(p["tier"]) == [0, 1, 1, 2, 2, 2]
    assert list(p["tiles"][:3]) == [0, 0, 0]
    t = nsgc.get_tune()
    tile = 1 << t.tile_log2
    for i in (3, 4, 5):
        assert p["tiles"][i] == -(-sizes[i] // tile)
        cls = int(np.floor(np.log2(sizes[i])))
        lt = t.cls[cls].link_target
        want = min(int(np.ceil(np.log2(max(1, -(-sizes[i] // lt))))), t.max_link_buckets_log2)
        # a wave target takes over when the window's row and column buckets
        # fit the wavefront kernel and its bucket count stays within the cap
        wt = t.cls[cls].wave_target
        if (wt > 0 and (1 << int(p["log2_row_buckets"][i])) <= 256
                and (1 << int(p["log2_col_buckets"][i])) <= 256):
            lw = int(np.ceil(np.log2(max(1, -(-sizes[i] // wt)))))
            if lw <= t.max_link_buckets_log2:
                want = lw
        assert p["log2_link_buckets"][i] == want
    assert p["workspace_bytes"] >= 24 * (sum(sizes[3:]))


def test_default_buckets_sized_by_their_tables():
    """Under the default tuning, a link bucket of a partitioned window below
    2^23 packets holds at most as many packets as its LDS table has slots (at
    2^23, twice as many), so it needs an overflow sweep only when nearly all
    its packets are distinct links, however the window's packets are spread.
    Row and column buckets hold at most twice as many packets as table slots
    below 2^19 packets and four times as many above (their ids, sources or
    destinations, repeat far more than links).  Wavefront buckets are checked
    against the wavefront table (2^9 slots)."""
    t = nsgc.default_tune()
    nsgc.set_tune(t)
    sizes = sorted({int(x) for x in np.unique(np.round(2.0 ** np.linspace(
        np.log2(t.small_max + 1), 23, 400)))} | {(1 << k) + d for k in range(11, 24)
                                                for d in (-1, 0, 1)} - {1 << 23 | 1})
    sizes = [n for n in sizes if t.small_max < n <= 1 << 23]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    p = nsgc.plan_inspect(off)
    assert (p["tier"] == 2).all()
    link_slots, rc_slots = 1 << t.link_slots_log2, 1 << t.rc_slots_log2
    for i, n in enumerate(sizes):
        lb, lr, lc = (int(p[k][i]) for k in ("log2_link_buckets", "log2_row_buckets",
                                             "log2_col_buckets"))
        cls = n.bit_length() - 1
        wave = (t.cls[cls].wave_target > 0 and lr <= 8 and lc <= 8
                and lb == int(np.ceil(np.log2(-(-n // t.cls[cls].wave_target)))))
        per_link = -(-n // (1 << lb))
        room = 512 if wave else link_slots
        assert per_link <= (room if n < 1 << 23 else 2 * room), (n, lb, wave)
        rc_room = (2 if n < 1 << 19 else 4) * rc_slots
        assert -(-n // (1 << lr)) <= rc_room, (n, lr)
        assert -(-n // (1 << lc)) <= rc_room, (n, lc)


def test_row_complete_plans_the_same_buckets_with_more_workspace():
    # row_complete changes how packets are spread over the link buckets, not
    # how many there are; its per-bucket source totals and per-window heavy
    # tables add workspace only when a wavefront window is present
    sizes = [500, 3000, 1 << 17, 1 << 21]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    before = nsgc.get_tune()
    try:
        nsgc.set_tune(nsgc.default_tune())
        q = nsgc.plan_inspect(off)
        base = nsgc.default_tune().to_dict()
        base["row_complete"] = 1
        nsgc.set_tune(nsgc.Tune.from_dict(base))
        p = nsgc.plan_inspect(off)
        for k in ("tier", "log2_link_buckets", "log2_row_buckets", "log2_col_buckets", "tiles"):
            assert (p[k] == q[k]).all(), k
        assert p["workspace_bytes"] > q["workspace_bytes"]
        big = np.array([0, 1 << 21], np.int64)   # workgroup windows only: nothing added
        assert nsgc.plan_inspect(big)["workspace_bytes"] == (
            nsgc.set_tune(nsgc.default_tune()) or nsgc.plan_inspect(big)["workspace_bytes"])
    finally:
        nsgc.set_tune(before)


def test_host_calls_from_many_threads():
    # host-only entry points called from several threads at once (ctypes
    # releases the GIL): tuning switches interleave with planning, and every
    # plan is one of the two tunings' plans
    import threading
    off = np.concatenate([[0], np.cumsum([3000, 1 << 17, 70000, 900, 1 << 20])]).astype(np.int64)
    before = nsgc.get_tune()
    a = nsgc.default_tune()
    b = nsgc.Tune.from_dict(dict(a.to_dict(), max_link_buckets_log2=8, tile_log2=12))
    try:
        nsgc.set_tune(a)
        want_a = nsgc.plan_inspect(off)
        nsgc.set_tune(b)
        want_b = nsgc.plan_inspect(off)
        assert (want_a["log2_link_buckets"] != want_b["log2_link_buckets"]).any()
        assert (want_a["tiles"] != want_b["tiles"]).any()
        errors = []

        def planner():
            for _ in range(200):
                got = nsgc.plan_inspect(off)
                if not any(all((got[k] == w[k]).all() for k in ("tier", "log2_link_buckets", "tiles"))
                           for w in (want_a, want_b)):
                    errors.append(got)

        def tuner():
            for i in range(400):
                nsgc.set_tune((a, b)[i % 2])
                nsgc.get_tune()

        threads = [threading.Thread(target=planner) for _ in range(4)] + [
            threading.Thread(target=tuner) for _ in range(2)]
        for t in threads:
            t.start()
        for t in threads:
            t.join(60)
        assert not any(t.is_alive() for t in threads)
        assert not errors
    finally:
        nsgc.set_tune(before)


def test_plan_rejects_bad_offsets():
    with pytest.raises(nsgc.NsgcError):
        nsgc.plan_inspect(np.array([0, 5, 2], np.int64))
    p = nsgc.plan_inspect(np.array([7], np.int64))
    assert p["tier"].size == 0


def test_plan_workspace_grows_with_packets():
    a = nsgc.plan_inspect(np.array([0, 1 << 16], np.int64))["workspace_bytes"]
    b = nsgc.plan_inspect(np.array([0, 1 << 20], np.int64))["workspace_bytes"]
    assert b > a >= 24 * (1 << 16)


def test_no_cpu_path():
    torch = pytest.importorskip("torch")
    s = torch.zeros(4, dtype=torch.int32)
    with pytest.raises(ValueError):
        nsgc.window_stats(s, s, [0, 4])


@pytest.mark.parametrize("tune", [
    {},
    {"cls": [[64, 64, 64]] * 33, "max_link_buckets_log2": 12, "max_rc_buckets_log2": 12,
     "small_max": 0},
    {"tile_log2": 11, "small_max": 0, "max_link_buckets_log2": 12},
    {"max_link_buckets_log2": 0, "max_rc_buckets_log2": 0, "small_max": 2048},
    {"cls": [[100, 300, 70]] * 33, "tile_log2": 13},
    {"row_complete": 1},
    {"row_complete": 1, "cls": [[2048, 4096, 4096, 64]] * 33, "max_link_buckets_log2": 12},
])
def test_plan_and_workspace_within_their_bounds(tune):
    # The graph form and nsgc_reserve size the plan buffer and the workspace
    # from bounds that depend only on the packet and window counts; every
    # batch of those counts must fit them.
    base = nsgc.default_tune().to_dict()
    base.update(tune)
    before = nsgc.get_tune()
    nsgc.set_tune(nsgc.Tune.from_dict(base))
    try:
        rng = np.random.default_rng(11)
        for trial in range(60):
            w = int(rng.integers(1, 300))
            kind = trial % 4
            if kind == 0:      # log-uniform, 1 .. 2^24
                sizes = np.floor(2.0 ** rng.uniform(0, 24, w)).astype(np.int64)
            elif kind == 1:    # just above powers of two times the targets
                sizes = (2 ** rng.integers(6, 22, w) + 1).astype(np.int64)
            elif kind == 2:    # one large window among empty and tiny ones
                sizes = rng.integers(0, 3, w).astype(np.int64)
                sizes[rng.integers(0, w)] = int(rng.integers(1 << 20, 1 << 25))
            else:              # all equal
                sizes = np.full(w, int(2 ** rng.uniform(8, 20)), np.int64)
            off = np.concatenate([[int(rng.integers(0, 1000))], sizes]).cumsum().astype(np.int64)
            s = nsgc.plan_sizes(off)
            assert 0 < s["plan_bytes"] <= s["plan_bound"], (tune, trial, s)
            assert 0 < s["workspace_bytes"] <= s["workspace_bound"], (tune, trial, s)
    finally:
        nsgc.set_tune(before)


def test_plain_mode_switch_is_host_state():
    assert nsgc.plain_mode() is False
    nsgc.set_plain_mode(True)
    try:
        assert nsgc.plain_mode() is True
    finally:
        nsgc.set_plain_mode(False)
    assert nsgc.plain_mode() is False


def test_reserve_rejects_negative_sizes_before_device_work():
    lib = nsgc.library()
    assert lib.nsgc_reserve(-1, 4) == -1
    assert lib.nsgc_reserve(4, -1) == -1
    assert lib.nsgc_reserve_stream(-1, 4, ctypes.c_void_p(0)) == -1
    assert lib.nsgc_reserve_stream(4, -1, ctypes.c_void_p(0)) == -1
