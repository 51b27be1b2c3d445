"""GPU parity: the HIP library against the CPU oracle, bit-exact on all nine
statistics (they are exact integer counts; the bar is equality).

Sizes here let the oracle finish in seconds while still spanning several
partition tiles, several link/row/column buckets and ragged tails.
"""
import numpy as np
import pytest

import oracle
import paper_2509_03653_amd as nsgc
import synth
from conftest import load_golden_batch, load_golden_windows
from gpu_util import assert_same, gpu_stats, say

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _default_tune():
    nsgc.set_tune(nsgc.default_tune())
    yield
    nsgc.set_tune(nsgc.default_tune())


def check(src, dst, off, what, forms=("batched",)):
    want = oracle.window_stats(src, dst, off, threads=8)
    for form in forms:
        say(f"[gpu] {what} form={form} windows={len(off) - 1} packets={int(off[-1] - off[0])}")
        assert_same(gpu_stats(src, dst, off, form), want, f"{what}/{form}")
    return want


def test_golden_windows_each_form():
    for name, (s, d, e) in sorted(load_golden_windows().items()):
        off = np.array([0, s.size], np.int64)
        for form in ("batched", "plain", "graph"):
            say(f"[gpu] golden {name} {form}")
            assert_same(gpu_stats(s, d, off, form), e[None, :], f"golden {name} {form}")


def test_golden_batch():
    src, dst, off, expected = load_golden_batch()
    for form in ("batched", "plain", "graph"):
        assert_same(gpu_stats(src, dst, off, form), expected, f"golden batch {form}")


def test_golden_windows_through_partitioned_tier():
    # the same hand-worked windows, forced through phases A-C (small tier off)
    t = nsgc.default_tune()
    t.small_max = 0
    nsgc.set_tune(t)
    for name, (s, d, e) in sorted(load_golden_windows().items()):
        off = np.array([0, s.size], np.int64)
        assert_same(gpu_stats(s, d, off), e[None, :], f"golden {name} partitioned")
    src, dst, off, expected = load_golden_batch()
    assert_same(gpu_stats(src, dst, off), expected, "golden batch partitioned")


def test_random_tiny_windows_many_alphabets():
    rng = np.random.default_rng(7)
    sizes = rng.integers(0, 300, 600)
    sizes[::50] = 0
    off = synth.offsets_from_sizes(sizes)
    n = int(off[-1])
    alph = rng.choice([1, 2, 3, 7, 40, 1000, 1 << 32], size=600)
    src = np.zeros(n, np.uint32)
    dst = np.zeros(n, np.uint32)
    for w in range(600):
        a, b = off[w], off[w + 1]
        src[a:b] = rng.integers(0, alph[w], b - a, dtype=np.uint64).astype(np.uint32)
        dst[a:b] = rng.integers(0, alph[w], b - a, dtype=np.uint64).astype(np.uint32)
        if w % 9 == 0:
            dst[a:b] = src[a:b]                   # self-loops
        if w % 13 == 0:
            src[a:b] = 0xFFFFFFFF                 # extreme addresses
            dst[a:(a + b) // 2] = 0xFFFFFFFF      # the packed key ~0 is legal
    check(src, dst, off, "tiny windows", forms=("batched", "plain", "graph"))


def test_size_boundaries():
    t = nsgc.get_tune()
    sm, tile = t.small_max, 1 << t.tile_log2
    sizes = [0, 1, 2, 63, 64, 65, sm - 1, sm, sm + 1, tile - 1, tile, tile + 1,
             2 * tile + 7, 5 * tile - 3, 3 * 2048 + 1]
    off = synth.offsets_from_sizes(sizes)
    rng = np.random.default_rng(11)
    n = int(off[-1])
    src = rng.integers(0, 300, n).astype(np.uint32)
    dst = rng.integers(0, 5000, n).astype(np.uint32)
    check(src, dst, off, "size boundaries", forms=("batched", "plain", "graph"))


def test_heavy_contention_windows():
    n = 40000
    off = synth.offsets_from_sizes([n, n, n, n, 700])
    src = np.zeros(int(off[-1]), np.uint32)
    dst = np.zeros(int(off[-1]), np.uint32)
    # w0: all packets identical
    src[0:n], dst[0:n] = 5, 9
    # w1: one source to many destinations (a star) plus repeats
    src[n:2 * n] = 77
    dst[n:2 * n] = np.arange(n) % 12345
    # w2: all packets are the key 0xFFFFFFFF_FFFFFFFF
    src[2 * n:3 * n] = 0xFFFFFFFF
    dst[2 * n:3 * n] = 0xFFFFFFFF
    # w3: address 0 and self-loops mixed
    rng = np.random.default_rng(3)
    x = rng.integers(0, 3, n).astype(np.uint32)
    src[3 * n:4 * n] = x
    dst[3 * n:4 * n] = np.where(rng.random(n) < 0.5, x, 0).astype(np.uint32)
    # w4: small window of identical packets
    src[4 * n:], dst[4 * n:] = 1, 1
    check(src, dst, off, "contention", forms=("batched", "plain"))


def test_wavefront_buckets_past_the_16_bit_counts():
    # The wavefront phase B keeps two 16-bit counts per word; a bucket of
    # 2^16 packets or more switches to half the slots with full-word counts.
    # Windows whose hot bucket holds exactly 2^16 - 1 packets (the last
    # narrow case), exactly 2^16, and far more, with and without other links.
    rng = np.random.default_rng(41)
    sizes = [65535, 65536, 1 << 17, 1 << 17, 1 << 18]
    off = synth.offsets_from_sizes(sizes)
    n = int(off[-1])
    src = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    dst = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    a = [int(x) for x in off]
    src[a[0]:a[1]], dst[a[0]:a[1]] = 3, 4            # one link, 65535 packets
    src[a[1]:a[2]], dst[a[1]:a[2]] = 3, 4            # one link, 65536 packets
    src[a[2]:a[3]], dst[a[2]:a[3]] = 0xFFFFFFFF, 7   # one link of 2^17 packets
    hot = a[3] + rng.choice(sizes[3], 70000, replace=False)
    src[hot], dst[hot] = 11, 12                      # 70000 packets among 61072 others
    hot = a[4] + rng.choice(sizes[4], 65535, replace=False)
    src[hot], dst[hot] = 13, 14                      # 65535 packets among 196609 others
    p = nsgc.plan_inspect(off)
    assert (p["tier"] == 2).all()
    # every window runs phase B one wavefront per 256-packet link bucket
    assert [int(x) for x in p["log2_link_buckets"]] == [
        int(np.ceil(np.log2(k / 256))) for k in sizes]
    check(src, dst, off, "16-bit count limit", forms=("batched", "graph", "noalloc"))


@pytest.mark.parametrize("maker", ["uniform_single", "zipf_batch", "skewed_large",
                                   "uneven_batch", "serving_stream"])
def test_workloads_scaled_down(maker):
    fn = synth.WORKLOADS[maker]
    if maker in ("uneven_batch", "serving_stream"):
        wl = fn(seed=2, num_windows=48, lo_log2=6, hi_log2=17)
    elif maker == "uniform_single":
        wl = fn(seed=2, num_windows=2, log2_window=17)
    else:
        wl = fn(seed=2, num_windows=6, log2_window=16)
    src, dst = wl.generate()
    check(src, dst, wl.offsets, maker, forms=("batched", "plain"))


@pytest.mark.parametrize("link_cap", [10, 12])
def test_large_window_short_segments(link_cap):
    # 2^21 packets cut into 128 tiles and 1024 (or more) link buckets leave
    # ~16 keys per (tile, bucket) segment and a few entries per (link bucket,
    # row bucket) segment: the gathers walk their segments concatenated
    wl = synth.uneven_batch(seed=6, num_windows=3, lo_log2=20, hi_log2=21)
    src, dst = wl.generate()
    base = nsgc.default_tune().to_dict()
    base.update(max_link_buckets_log2=link_cap)
    nsgc.set_tune(nsgc.Tune.from_dict(base))
    check(src, dst, wl.offsets, f"large windows link cap 2^{link_cap}")


@pytest.mark.parametrize("windows", [256, 257])
def test_phase_c_order_limit(windows):
    # 2^17-packet windows have 32 row and 32 column buckets: 256 windows give
    # exactly 16384 phase-C items (taken largest first), 257 windows one
    # window more (taken in their own order)
    wl = synth.zipf_batch(seed=8, num_windows=windows, log2_window=17)
    p = nsgc.plan_inspect(wl.offsets)
    assert int(np.sum((1 << p["log2_row_buckets"]) + (1 << p["log2_col_buckets"]))) == 64 * windows
    src, dst = wl.generate()
    check(src, dst, wl.offsets, f"{windows} x 2^17 (phase-C order limit)")


TUNES = {
    "tiny_tables_forced_sweeps": dict(link_slots_log2=10, rc_slots_log2=10,
                                      cls=[[65536, 65536, 65536]] * 33),
    "small_tier_off": dict(small_max=0),
    "small_tier_max": dict(small_max=2048),
    "tile_2k": dict(tile_log2=11),
    "tile_16k": dict(tile_log2=14),
    "one_bucket": dict(max_link_buckets_log2=0, max_rc_buckets_log2=0),
    "many_buckets": dict(cls=[[64, 64, 64]] * 33, max_link_buckets_log2=12,
                         max_rc_buckets_log2=12),
    "big_tables": dict(link_slots_log2=12, rc_slots_log2=13, blocks_per_cu=1),
    # per-id combining in phase B, and its fallback (gives up almost always)
    "combine": dict(combine_probes=64),
    "combine_fallback": dict(combine_probes=1),
    "combine_fallback_tight": dict(combine_probes=2, link_slots_log2=10,
                                   cls=[[512, 4096, 4096]] * 33),
    # phase B one wavefront per bucket: off, tiny buckets, and buckets far
    # beyond the wavefront table (overflow sweeps inside a wavefront)
    "workgroup_phase_b": dict(cls=[[2048, 4096, 4096, 0]] * 33),
    "wave_tiny_buckets": dict(cls=[[2048, 4096, 4096, 64]] * 33, max_link_buckets_log2=12),
    "wave_forced_sweeps": dict(cls=[[2048, 4096, 4096, 2048]] * 33),
    "wave_many_rc_buckets": dict(cls=[[2048, 256, 256, 128]] * 33, max_link_buckets_log2=12,
                                 max_rc_buckets_log2=12),
}


@pytest.mark.parametrize("name", sorted(TUNES))
def test_every_tuning_gives_identical_results(name):
    wl = synth.zipf_batch(seed=4, num_windows=5, log2_window=15)
    src, dst = wl.generate()
    sizes = [0, 1, 900, 3000, 20000, 1 << 15, 77777]
    off = synth.offsets_from_sizes(sizes)
    s2, d2 = synth.fill(off, 9, wl.src_dist, wl.dst_dist)
    base = nsgc.default_tune().to_dict()
    base.update(TUNES[name])
    nsgc.set_tune(nsgc.Tune.from_dict(base))
    check(src, dst, wl.offsets, f"tune {name} zipf")
    check(s2, d2, off, f"tune {name} mixed sizes", forms=("batched", "plain"))


def test_wavefront_and_workgroup_windows_in_one_batch():
    # windows up to 2^19 packets take link aggregation one wavefront per bucket
    # (under the default tuning), larger ones one workgroup per bucket; both
    # kernels draw their items from their own list of the batch's phase-B items
    sizes = [5000, 300000, 70000, 1 << 19, 1500, 0, 2000, 600000, 262145, 40000,
             (1 << 20) + 3]
    off = synth.offsets_from_sizes(sizes)
    wl = synth.zipf_batch(seed=3, num_windows=1, log2_window=4)
    src, dst = synth.fill(off, 12, wl.src_dist, wl.dst_dist)
    p = nsgc.plan_inspect(off)
    t = nsgc.get_tune()
    wave = [sizes[i] > t.small_max and int(p["log2_link_buckets"][i]) > int(
        np.ceil(np.log2(-(-sizes[i] // t.cls[int(np.log2(sizes[i]))].link_target))))
        for i in range(len(sizes)) if sizes[i] > 0]
    assert any(wave) and not all(wave)
    check(src, dst, off, "wavefront and workgroup windows", forms=("batched", "plain", "graph"))


def test_addresses_hashed_to_the_empty_marker():
    # the source and destination whose hashed forms equal the tables' empty
    # marker (and their link, whose key is the 64-bit marker) are counted
    # outside the tables, in every tier and phase-B kernel
    from hashed_addresses import DESTINATION_MARKER, SOURCE_MARKER
    rng = np.random.default_rng(17)
    sizes = [7, 900, 5000, 300000, 1500, 70000]
    off = synth.offsets_from_sizes(sizes)
    n = int(off[-1])
    pool = np.array([SOURCE_MARKER, DESTINATION_MARKER, 0, 0xFFFFFFFF, 5, 6], np.uint32)
    src = pool[rng.integers(0, pool.size, n)]
    dst = pool[rng.integers(0, pool.size, n)]
    src[::3] = SOURCE_MARKER
    dst[::3] = DESTINATION_MARKER
    wide = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    src[1::4] = wide[1::4]                   # enough distinct links for the larger tiers
    for form in ("batched", "plain", "graph"):
        check(src, dst, off, "marker addresses", forms=(form,))
    for name, extra in (("workgroup", dict(cls=[[2048, 4096, 4096, 0]] * 33)),
                        ("sweeps", dict(link_slots_log2=10, rc_slots_log2=10,
                                        cls=[[65536, 65536, 65536, 2048]] * 33))):
        base = nsgc.default_tune().to_dict()
        base.update(extra)
        nsgc.set_tune(nsgc.Tune.from_dict(base))
        check(src, dst, off, f"marker addresses, {name}")


def test_repeated_runs_identical_and_nonzero_first_offset():
    wl = synth.uneven_batch(seed=5, num_windows=30, lo_log2=8, hi_log2=16)
    src, dst = wl.generate()
    off = wl.offsets + 0
    # drop the first 123 packets from window 0 so offsets[0] is non-zero
    off[0] = 123
    want = oracle.window_stats(src, dst, off, threads=8)
    first = gpu_stats(src, dst, off)
    assert_same(first, want, "offset start")
    for _ in range(4):
        assert_same(gpu_stats(src, dst, off), first, "repeat")


def test_window_alone_equals_window_in_batch():
    wl = synth.uneven_batch(seed=6, num_windows=20, lo_log2=8, hi_log2=16)
    src, dst = wl.generate()
    batch = gpu_stats(src, dst, wl.offsets)
    for w in (0, 7, 19):
        a, b = int(wl.offsets[w]), int(wl.offsets[w + 1])
        alone = gpu_stats(src[a:b], dst[a:b], np.array([0, b - a], np.int64))
        assert_same(alone[0:1], batch[w:w + 1], f"alone w{w}")


def test_graph_reuse_with_different_batches():
    import torch
    g = nsgc.Graph(1 << 18, 64)
    try:
        for seed, nw in ((1, 40), (2, 3), (3, 64), (4, 1)):
            wl = synth.uneven_batch(seed=seed, num_windows=nw, lo_log2=4, hi_log2=12)
            src, dst = wl.generate()
            want = oracle.window_stats(src, dst, wl.offsets)
            got = gpu_stats(src, dst, wl.offsets, "graph", graph=g)
            assert_same(got, want, f"graph reuse seed {seed}")
        torch.cuda.synchronize()
    finally:
        g.close()


def test_graph_plan_holds_many_items_per_window():
    # tiny bucket targets and the largest bucket cap give thousands of phase-B
    # and phase-C items per window: the graph's plan buffer, sized when the
    # graph is created, must hold their per-item tables
    import torch
    base = nsgc.default_tune().to_dict()
    base.update(cls=[[64, 64, 64]] * 33, max_link_buckets_log2=12, max_rc_buckets_log2=12,
                small_max=0)
    nsgc.set_tune(nsgc.Tune.from_dict(base))
    g = nsgc.Graph(1 << 20, 4)
    try:
        for seed, sizes in ((1, [1 << 18, 1 << 18, 1 << 18, 1 << 18]), (2, [1 << 20]),
                            (3, [5, 1 << 19, 3, (1 << 19) - 8])):
            off = synth.offsets_from_sizes(sizes)
            wl = synth.zipf_batch(seed=seed, num_windows=1, log2_window=4)
            src, dst = synth.fill(off, seed, wl.src_dist, wl.dst_dist)
            want = oracle.window_stats(src, dst, off, threads=4)
            say(f"[gpu] graph, many items per window, seed {seed}")
            assert_same(gpu_stats(src, dst, off, "graph", graph=g), want, f"many items {seed}")
        torch.cuda.synchronize()
    finally:
        g.close()


def test_stream_argument_and_out_reuse():
    import torch
    wl = synth.zipf_batch(seed=8, num_windows=3, log2_window=14)
    src, dst = wl.generate()
    want = oracle.window_stats(src, dst, wl.offsets)
    s = torch.from_numpy(src.view(np.int32)).cuda()
    d = torch.from_numpy(dst.view(np.int32)).cuda()
    out = torch.full((3, 9), -1, dtype=torch.int64, device="cuda")
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    nsgc.window_stats(s, d, wl.offsets, out=out, stream=st)
    st.synchronize()
    assert_same(out.cpu().numpy().view(np.uint64), want, "side stream")


def test_concurrent_host_threads_on_their_own_streams():
    # host threads plan and enqueue at the same time, each on its own stream
    # (a lock per stream), while another thread switches the tuning (which
    # never changes a result); every call must return the oracle's statistics
    import threading

    import torch
    cases = []
    for seed, windows, log2 in ((21, 5, 15), (22, 9, 13), (23, 2, 17)):
        wl = synth.zipf_batch(seed=seed, num_windows=windows, log2_window=log2)
        src, dst = wl.generate()
        cases.append((torch.from_numpy(src.view(np.int32)).cuda(),
                      torch.from_numpy(dst.view(np.int32)).cuda(), wl.offsets,
                      oracle.window_stats(src, dst, wl.offsets, threads=8)))
    torch.cuda.synchronize()
    errors = []
    stop = threading.Event()

    def worker(k):
        s, d, off, want = cases[k]
        st = torch.cuda.Stream()
        try:
            for it in range(25):
                out = torch.full((len(off) - 1, 9), -1, dtype=torch.int64, device="cuda")
                fn = (nsgc.window_stats, nsgc.window_stats_plain)[it % 5 == 4]
                fn(s, d, off, out=out, stream=st)
                st.synchronize()
                got = out.cpu().numpy().view(np.uint64)
                if not np.array_equal(got, want):
                    errors.append((k, it))
        except Exception as e:   # reported below, on the main thread
            errors.append((k, repr(e)))

    def tuner():
        a = nsgc.default_tune()
        b = nsgc.Tune.from_dict(dict(a.to_dict(), blocks_per_cu=2, small_max=512))
        i = 0
        while not stop.is_set():
            nsgc.set_tune((a, b)[i % 2])
            i += 1

    say("[gpu] three threads on three streams, one switching the tuning")
    threads = [threading.Thread(target=worker, args=(k,)) for k in range(len(cases))]
    tt = threading.Thread(target=tuner)
    tt.start()
    for t in threads:
        t.start()
    for t in threads:
        t.join(120)
    stop.set()
    tt.join(10)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors


def test_heavy_links_split_entries():
    # links with more packets than an emission entry's packet field holds
    # (2^19 - 1) are emitted as several entries; every path must sum them
    n = 1_300_000
    rng = np.random.default_rng(31)
    src = rng.integers(0, 50, n).astype(np.uint32)
    dst = rng.integers(0, 50, n).astype(np.uint32)
    src[: 600_000], dst[: 600_000] = 1, 2          # one link of 600K packets
    src[600_000: 1_200_000] = 1                    # source 1: 1.2M packets
    dst[600_000: 1_200_000] = 3
    perm = rng.permutation(n)
    src, dst = src[perm], dst[perm]
    off = synth.offsets_from_sizes([n, 1000, n // 2])
    s2 = np.concatenate([src, src[:1000], src[: n // 2]])
    d2 = np.concatenate([dst, dst[:1000], dst[: n // 2]])
    check(s2, d2, off, "heavy links", forms=("batched", "plain"))
    one = dict(max_link_buckets_log2=0, max_rc_buckets_log2=0)
    for extra in (one, dict(combine_probes=1), dict(combine_probes=64),
                  dict(link_slots_log2=10, **one)):   # overflow sweeps
        base = nsgc.default_tune().to_dict()
        base.update(extra)
        nsgc.set_tune(nsgc.Tune.from_dict(base))
        check(s2, d2, off, f"heavy links {extra}")


def test_abandoned_bucket_is_reported_not_hung():
    # With no overflow sweeps allowed, a bucket whose LDS table overflows is
    # abandoned: its window must come back marked invalid (bit 63 of stat 0)
    # while the other windows of the batch stay exact.
    rng = np.random.default_rng(21)
    sizes = [3000, 9000, 9000, 2500]
    off = synth.offsets_from_sizes(sizes)
    n = int(off[-1])
    src = np.zeros(n, np.uint32)
    dst = np.zeros(n, np.uint32)
    a = [int(x) for x in off]
    src[a[0]:a[1]] = rng.integers(0, 10, sizes[0])          # few links: fits
    dst[a[0]:a[1]] = rng.integers(0, 5, sizes[0])
    src[a[1]:a[2]] = np.arange(sizes[1]) * 7 + 1            # 9000 distinct links
    dst[a[1]:a[2]] = np.arange(sizes[1]) % 97
    src[a[2]:a[3]] = 5                                       # 3000 distinct columns
    dst[a[2]:a[3]] = np.arange(sizes[2]) % 3000
    src[a[3]:a[4]] = rng.integers(0, 40, sizes[3])
    dst[a[3]:a[4]] = rng.integers(0, 40, sizes[3])
    want = oracle.window_stats(src, dst, off)
    base = nsgc.default_tune().to_dict()
    base.update(link_slots_log2=12, rc_slots_log2=10, max_sweeps_log2=0, small_max=1024,
                cls=[[1 << 20, 1 << 20, 1 << 20]] * 33,
                max_link_buckets_log2=0, max_rc_buckets_log2=0)
    nsgc.set_tune(nsgc.Tune.from_dict(base))
    for form in ("batched", "plain"):
        say(f"[gpu] abandoned buckets form={form}")
        got = gpu_stats(src, dst, off, form)
        marked = (got[:, 0] >> np.uint64(63)) != 0
        # w1: 9000 distinct links overflow the 4096-slot link table;
        # w2: 3000 distinct destinations overflow the 1024-slot column table
        assert list(marked) == [False, True, True, False], got
        assert_same(got[[0, 3]], want[[0, 3]], f"unaffected windows {form}")
        with pytest.raises(nsgc.NsgcError):
            nsgc.check_valid(got)
    # the default sweep limit handles the same batch exactly
    nsgc.set_tune(nsgc.default_tune())
    assert_same(gpu_stats(src, dst, off), want, "default sweeps")


def test_plain_mode_routes_the_batched_entry_point():
    rng = np.random.default_rng(31)
    sizes = [0, 5, 3000, 70000, 1]
    off = synth.offsets_from_sizes(sizes)
    n = int(off[-1])
    src = rng.integers(0, 300, n).astype(np.uint32)
    dst = rng.integers(0, 900, n).astype(np.uint32)
    want = oracle.window_stats(src, dst, off)
    nsgc.set_plain_mode(True)
    try:
        say("[gpu] plain mode through nsgc_window_stats")
        assert_same(gpu_stats(src, dst, off, "batched"), want, "plain mode")
    finally:
        nsgc.set_plain_mode(False)
    assert_same(gpu_stats(src, dst, off, "batched"), want, "batched mode")


def test_direct_forms_refuse_a_capturing_stream():
    # A direct call inside a stream capture returns NSGC_ERR_CAPTURING with
    # nothing enqueued; the capture itself stays valid and ends normally.
    import ctypes
    import torch
    from gpu_util import to_gpu
    s = to_gpu(np.arange(4096, dtype=np.uint32))
    off = np.array([0, 2048, 4096], np.int64)
    out = torch.full((2, 9), -7, dtype=torch.int64, device="cuda")
    lib = nsgc.library()
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("[gpu] direct forms under capture")
    codes = []
    with torch.cuda.graph(g, stream=stream):
        h = ctypes.c_void_p(int(stream.cuda_stream))
        for fn in (lib.nsgc_window_stats, lib.nsgc_window_stats_plain):
            codes.append(fn(ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(s.data_ptr()),
                            ctypes.c_void_p(off.ctypes.data), 2, ctypes.c_void_p(out.data_ptr()), h))
        codes.append(lib.nsgc_reserve_stream(1 << 20, 16, h))
        out.add_(0)                     # keep the captured graph non-empty
    assert codes == [-6, -6, -6], codes
    g.replay()
    torch.cuda.synchronize()
    assert bool((out == -7).all())      # nothing was enqueued into the graph


def test_graph_launches_on_two_streams_are_serialised():
    # One graph object launched alternately on two streams: every launch must
    # see its own batch (the instances share one workspace).
    import torch
    from gpu_util import to_gpu
    wl = synth.zipf_batch(seed=5, num_windows=6, log2_window=15)
    src, dst = wl.generate()
    off = wl.offsets
    want = oracle.window_stats(src, dst, off, threads=8)
    rev = np.ascontiguousarray(dst), np.ascontiguousarray(src)
    want_rev = oracle.window_stats(rev[0], rev[1], off, threads=8)
    g = nsgc.Graph(int(off[-1]), len(off) - 1)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    s1, d1 = to_gpu(src), to_gpu(dst)
    outs = []
    say("[gpu] graph on two streams")
    for i in range(6):
        a, b = (s1, d1) if i % 2 == 0 else (d1, s1)
        outs.append(g.launch(a, b, off, stream=streams[i % 2]))
    torch.cuda.synchronize()
    g.close()
    for i, o in enumerate(outs):
        assert_same(o.cpu().numpy().view(np.uint64), want if i % 2 == 0 else want_rev,
                    f"launch {i}")
