"""GPU parity of the row-complete partition (tune row_complete = 1).

Light sources keep all their links in one link bucket, whose phase-B
wavefront then gives their packets and fan-out itself; sources that a sample
of the window shows to be heavy are spread over the other buckets and leave
one combined entry per bucket for phase C.  Every case is compared bit for
bit with the oracle: heavy sources split across buckets, a heavy source that
the sample misses (its bucket overflows and sweeps), more sources per bucket
than the row table holds, two-bucket windows, the all-ones hashed ids, and
every entry-point form.
"""
import numpy as np
import pytest

import oracle
import paper_2509_03653_amd as nsgc
import synth
from gpu_util import assert_same, gpu_stats, say

pytestmark = pytest.mark.gpu

SAMPLE, RUN = 4096, 256   # the heavy-source sample: 16 runs of 256 packets


@pytest.fixture(autouse=True)
def _row_complete():
    nsgc.set_tune(_tune())
    yield
    nsgc.set_tune(nsgc.default_tune())


def _tune(**extra):
    base = nsgc.default_tune().to_dict()
    base["row_complete"] = 1
    base.update(extra)
    return nsgc.Tune.from_dict(base)


def check(src, dst, off, what, forms=("batched",)):
    want = oracle.window_stats(src, dst, off, threads=8)
    for form in forms:
        say(f"[gpu] rows {what} form={form} windows={len(off) - 1} packets={int(off[-1] - off[0])}")
        assert_same(gpu_stats(src, dst, off, form), want, f"rows {what}/{form}")
    return want


def _sampled(n):
    """Positions of a window of n packets that the heavy-source sample reads."""
    if n <= SAMPLE:
        return np.arange(n)
    return np.concatenate([np.arange(RUN) + (n - RUN) * j // 15 for j in range(16)])


def test_zipf_batch_every_form():
    wl = synth.zipf_batch(seed=5, num_windows=6, log2_window=16)
    src, dst = wl.generate()
    check(src, dst, wl.offsets, "zipf 6 x 2^16", forms=("batched", "plain", "graph", "noalloc"))


def test_dominant_sources_split_across_buckets():
    # sources with 40%, 10% and 2% of each window and many destinations each,
    # over a Zipf background; windows of 2 .. 2^10 link buckets
    rng = np.random.default_rng(7)
    sizes = [1100, 2048, 9000, 1 << 16, 200_000]
    off = synth.offsets_from_sizes(sizes)
    wl = synth.zipf_batch(seed=8, num_windows=1, log2_window=4)
    src, dst = synth.fill(off, 21, wl.src_dist, wl.dst_dist)
    for w in range(len(sizes)):
        a, b = int(off[w]), int(off[w + 1])
        u = rng.random(b - a)
        s = src[a:b]
        s[u < 0.40] = 7
        s[(u >= 0.40) & (u < 0.50)] = 8
        s[(u >= 0.50) & (u < 0.52)] = 9
        dst[a:b][u < 0.52] = rng.integers(0, 1 << 20, int(np.sum(u < 0.52))).astype(np.uint32)
    check(src, dst, off, "dominant sources", forms=("batched", "graph"))


def test_single_source_window():
    # one source, every destination distinct: the whole window is one heavy row
    n = 1 << 17
    src = np.full(n, 12345, np.uint32)
    dst = np.arange(n, dtype=np.uint32) * np.uint32(2654435761)
    off = np.array([0, n], np.int64)
    check(src, dst, off, "single source")


def test_heavy_source_missed_by_the_sample():
    # a source with a quarter of the window's packets, all at positions the
    # sample does not read: it counts as light, its bucket overflows the
    # wavefront table and sweeps, and the bucket falls back to per-link rows
    n = 1 << 17
    rng = np.random.default_rng(11)
    wl = synth.zipf_batch(seed=9, num_windows=1, log2_window=17)
    src, dst = wl.generate()
    free = np.setdiff1d(np.arange(n), _sampled(n))
    pick = rng.choice(free, n // 4, replace=False)
    src[pick] = 424242
    dst[pick] = rng.integers(0, 1 << 24, pick.size).astype(np.uint32)
    check(src, dst, wl.offsets, "missed heavy source", forms=("batched", "plain"))


def test_more_sources_than_the_row_table_holds():
    # buckets of 2048 packets with nearly all sources distinct: the row table
    # (256 slots) overflows and the bucket keeps per-link row entries
    rng = np.random.default_rng(13)
    sizes = [1 << 15, 1 << 16, 5000]
    off = synth.offsets_from_sizes(sizes)
    n = int(off[-1])
    src = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    dst = rng.integers(0, 64, n).astype(np.uint32)
    for wave in (1024, 2048):
        nsgc.set_tune(_tune(cls=[[2048, 4096, 4096, wave]] * 33))
        check(src, dst, off, f"row table overflow wave_target={wave}")


def test_tuning_variants():
    wl = synth.zipf_batch(seed=4, num_windows=5, log2_window=15)
    src, dst = wl.generate()
    sizes = [0, 1, 300, 512, 900, 1025, 3000, 20000, 1 << 15, 77777, 300000]   # 300, 512:
    # two link buckets when the small tier is off
    off = synth.offsets_from_sizes(sizes)
    s2, d2 = synth.fill(off, 9, wl.src_dist, wl.dst_dist)
    for name, extra in (("tiny buckets", dict(cls=[[2048, 4096, 4096, 64]] * 33,
                                              max_link_buckets_log2=12)),
                        ("forced sweeps", dict(cls=[[2048, 4096, 4096, 2048]] * 33)),
                        ("many rc buckets", dict(cls=[[2048, 256, 256, 128]] * 33,
                                                 max_link_buckets_log2=12,
                                                 max_rc_buckets_log2=12)),
                        ("tile 2k", dict(tile_log2=11)),
                        ("small tier off", dict(small_max=0))):
        nsgc.set_tune(_tune(**extra))
        check(src, dst, wl.offsets, f"{name} zipf")
        check(s2, d2, off, f"{name} mixed sizes", forms=("batched", "plain"))


def test_addresses_hashed_to_the_empty_marker():
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
    src[1::4] = wide[1::4]
    dst[2::5] = wide[2::5]
    check(src, dst, off, "marker addresses", forms=("batched", "graph"))
    # the marker source as a light source (few packets): home bucket only
    src2 = wide.copy()
    src2[5:40] = SOURCE_MARKER
    check(src2, dst, off, "light marker source")


def test_benchmark_shape():
    # the benchmark's window size and source skew, 16 windows in full
    wl = synth.zipf_batch(seed=2, num_windows=16, log2_window=17)
    src, dst = wl.generate()
    check(src, dst, wl.offsets, "zipf 16 x 2^17", forms=("batched", "graph"))
