"""Pins for the CPU oracle: each test ties it to something other than itself.

* hand-worked windows from Table III's definitions (tests/golden/);
* closed forms for structured windows;
* exact invariants that relate the nine statistics;
* metamorphic relations (packet order, injective relabelling -- the paper's
  anonymisation is a bijection on addresses, Section IV "IP Address
  Anonymization" --, the src/dst swap of Table III's caption, repetition,
  disjoint union);
* an O(n^2) brute force on tiny windows and a numpy.unique formulation on
  medium windows (tests/independent_refs.py).

A plausible slip in the oracle (a dropped term, rows and columns swapped,
fan-out counted as packets, max over the wrong view, an off-by-one in the
window bounds) fails at least one of these.
"""
import numpy as np
import pytest

import oracle
import synth
from conftest import load_golden_batch, load_golden_windows
from independent_refs import brute_force, numpy_unique

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def one(src, dst):
    src = np.asarray(src, dtype=np.uint32)
    dst = np.asarray(dst, dtype=np.uint32)
    off = np.array([0, src.size], dtype=np.int64)
    return oracle.window_stats(src, dst, off)[0]


# ---------------------------------------------------------------- golden ----

@pytest.mark.parametrize("name", sorted(load_golden_windows().keys()))
def test_hand_worked_window(name):
    src, dst, expected = load_golden_windows()[name]
    np.testing.assert_array_equal(one(src, dst), expected)


def test_hand_worked_batch():
    src, dst, offsets, expected = load_golden_batch()
    got = oracle.window_stats(src, dst, offsets)
    np.testing.assert_array_equal(got, expected)
    got_mt = oracle.window_stats(src, dst, offsets, threads=3)
    np.testing.assert_array_equal(got_mt, expected)


def test_nonzero_first_offset_and_gaps():
    # offsets[0] may be non-zero; packets outside every window are ignored
    wins = load_golden_windows()
    s1, d1, e1 = wins["ex1"]
    s7, d7, e7 = wins["ex7"]
    junk = np.array([99, 98, 97], dtype=np.uint32)
    src = np.concatenate([junk, s1, junk, s7])
    dst = np.concatenate([junk, d1, junk, d7])
    off = np.array([3, 3 + s1.size], dtype=np.int64)
    np.testing.assert_array_equal(oracle.window_stats(src, dst, off)[0], e1)
    off = np.array([6 + s1.size, 6 + s1.size + s7.size], dtype=np.int64)
    np.testing.assert_array_equal(oracle.window_stats(src, dst, off)[0], e7)


def test_rejects_bad_offsets():
    src = np.zeros(4, np.uint32)
    with pytest.raises(ValueError):
        oracle.window_stats(src, src, np.array([0, 3, 2], np.int64))
    with pytest.raises(ValueError):
        oracle.window_stats(src, src, np.array([-1, 2], np.int64))
    assert oracle.window_stats(src, src, np.array([0], np.int64)).shape == (0, 9)


# ----------------------------------------------------------- closed forms ----

@pytest.mark.parametrize("n", [1, 2, 17, 1000])
def test_all_identical(n):
    s = np.full(n, 5, np.uint32)
    d = np.full(n, 6, np.uint32)
    np.testing.assert_array_equal(one(s, d), [n, 1, n, 1, n, 1, 1, n, 1])


@pytest.mark.parametrize("n", [1, 3, 500])
def test_bijection(n):
    rng = np.random.default_rng(n)
    s = rng.permutation(10 * n)[:n].astype(np.uint32)
    d = rng.permutation(10 * n)[:n].astype(np.uint32) + np.uint32(7)
    np.testing.assert_array_equal(one(s, d), [n, n, 1, n, 1, 1, n, 1, 1])


@pytest.mark.parametrize("n", [1, 2, 300])
def test_star(n):
    s = np.full(n, 42, np.uint32)
    d = np.arange(n, dtype=np.uint32) * np.uint32(3) + np.uint32(1)
    np.testing.assert_array_equal(one(s, d), [n, n, 1, 1, n, n, n, 1, 1])
    # the reverse star: many sources into one destination
    np.testing.assert_array_equal(one(d, s), [n, n, 1, n, 1, 1, 1, n, n])


@pytest.mark.parametrize("k,m,t", [(1, 1, 1), (3, 5, 1), (7, 2, 1), (4, 6, 3), (5, 5, 7)])
def test_complete_bipartite(k, m, t):
    ss, dd = np.meshgrid(np.arange(k) + 100, np.arange(m) + 1000, indexing="ij")
    s = np.repeat(ss.ravel(), t).astype(np.uint32)
    d = np.repeat(dd.ravel(), t).astype(np.uint32)
    rng = np.random.default_rng(k * 31 + m)
    p = rng.permutation(s.size)
    got = one(s[p], d[p])
    np.testing.assert_array_equal(got, [t * k * m, k * m, t, k, t * m, m, m, t * k, k])


# -------------------------------------------------------------- invariants ---

def check_invariants(st, n):
    v, l, ml, us, ms, fo, ud, md, fi = [int(x) for x in st]
    assert v == n
    assert l <= n
    if n == 0:
        assert all(int(x) == 0 for x in st)
        return
    assert all(int(x) >= 1 for x in st)
    assert max(us, ud) <= l <= us * ud
    assert fo <= ud and fi <= us
    assert ml <= min(ms, md)
    assert fo <= ms and fi <= md
    assert ms * us >= v and md * ud >= v
    assert fo * us >= l and fi * ud >= l


def _small_workload(seed, windows=24):
    wl = synth.zipf_batch(seed=seed, num_windows=windows, log2_window=10)
    src, dst = wl.generate()
    return src, dst, wl.offsets


def test_invariants_on_synthetic_windows():
    for seed in (1, 2, 3):
        src, dst, off = _small_workload(seed)
        got = oracle.window_stats(src, dst, off, threads=4)
        for w in range(len(off) - 1):
            check_invariants(got[w], int(off[w + 1] - off[w]))


def test_sums_of_vectors_match_scalars():
    # sum r = sum c = valid packets, sum f = sum g = unique links
    src, dst, off = _small_workload(7, windows=4)
    st = oracle.window_stats(src, dst, off)
    for w in range(4):
        e = oracle.window_entities(src, dst, int(off[w]), int(off[w + 1]))
        assert int(e["row_packets"].sum()) == int(st[w, 0]) == int(e["col_packets"].sum())
        assert int(e["row_links"].sum()) == int(st[w, 1]) == int(e["col_links"].sum())
        assert int(e["link_counts"].sum()) == int(st[w, 0])
        assert e["link_keys"].size == int(st[w, 1])
        assert e["row_ids"].size == int(st[w, 3]) and e["col_ids"].size == int(st[w, 6])


# ------------------------------------------------------------- metamorphic ---

def test_packet_order_does_not_matter():
    src, dst, off = _small_workload(11, windows=3)
    base = oracle.window_stats(src, dst, off)
    rng = np.random.default_rng(0)
    s2, d2 = src.copy(), dst.copy()
    for w in range(3):
        a, b = int(off[w]), int(off[w + 1])
        p = rng.permutation(b - a) + a
        s2[a:b], d2[a:b] = src[p], dst[p]
    np.testing.assert_array_equal(oracle.window_stats(s2, d2, off), base)


def test_injective_relabelling_does_not_matter():
    # anonymisation maps every address through one bijection
    src, dst, off = _small_workload(12, windows=3)
    base = oracle.window_stats(src, dst, off)
    relabel = np.vectorize(lambda x: synth.pool_address(int(x), 0x1234567), otypes=[np.uint32])
    np.testing.assert_array_equal(oracle.window_stats(relabel(src), relabel(dst), off), base)
    # independent bijections on the two columns also leave everything unchanged
    relabel2 = np.vectorize(lambda x: synth.pool_address(int(x), 0x7654321), otypes=[np.uint32])
    np.testing.assert_array_equal(oracle.window_stats(relabel(src), relabel2(dst), off), base)


def test_swapping_src_and_dst_swaps_the_views():
    src, dst, off = _small_workload(13, windows=3)
    a = oracle.window_stats(src, dst, off)
    b = oracle.window_stats(dst, src, off)
    np.testing.assert_array_equal(b[:, 0:3], a[:, 0:3])
    np.testing.assert_array_equal(b[:, 3:6], a[:, 6:9])
    np.testing.assert_array_equal(b[:, 6:9], a[:, 3:6])


@pytest.mark.parametrize("t", [2, 5])
def test_repeating_a_window(t):
    src, dst, off = _small_workload(14, windows=2)
    for w in range(2):
        s, d = src[off[w]:off[w + 1]], dst[off[w]:off[w + 1]]
        a = one(s, d).astype(np.int64)
        b = one(np.tile(s, t), np.tile(d, t)).astype(np.int64)
        scaled = a.copy()
        scaled[[0, 2, 4, 7]] *= t
        np.testing.assert_array_equal(b, scaled)


def test_disjoint_union():
    s1 = np.array([1, 1, 2, 3, 3, 3], np.uint32); d1 = np.array([5, 6, 5, 5, 5, 7], np.uint32)
    s2 = np.array([10, 11, 11, 11], np.uint32); d2 = np.array([20, 20, 21, 21], np.uint32)
    a, b = one(s1, d1).astype(np.int64), one(s2, d2).astype(np.int64)
    u = one(np.concatenate([s1, s2]), np.concatenate([d1, d2])).astype(np.int64)
    summed = [0, 1, 3, 6]
    maxed = [2, 4, 5, 7, 8]
    np.testing.assert_array_equal(u[summed], a[summed] + b[summed])
    np.testing.assert_array_equal(u[maxed], np.maximum(a[maxed], b[maxed]))


def test_batch_composition_does_not_matter():
    src, dst, off = _small_workload(15, windows=6)
    whole = oracle.window_stats(src, dst, off)
    for w in range(6):
        alone = oracle.window_stats(src[off[w]:off[w + 1]], dst[off[w]:off[w + 1]],
                                    np.array([0, off[w + 1] - off[w]], np.int64))
        np.testing.assert_array_equal(alone[0], whole[w])


# --------------------------------------------------- independent references ---

def test_brute_force_matches_golden():
    for name, (s, d, e) in load_golden_windows().items():
        np.testing.assert_array_equal(brute_force(s, d), e, err_msg=name)
        np.testing.assert_array_equal(numpy_unique(s, d), e, err_msg=name)


def test_oracle_vs_brute_force_tiny_windows():
    rng = np.random.default_rng(2024)
    checked = 0
    for trial in range(3000):
        n = int(rng.integers(0, 96)) if trial % 10 else int(rng.integers(96, 400))
        alphabet = int(rng.choice([1, 2, 3, 5, 8, 20, 1000, 2 ** 32]))
        s = rng.integers(0, alphabet, n, dtype=np.uint64).astype(np.uint32)
        d = rng.integers(0, alphabet, n, dtype=np.uint64).astype(np.uint32)
        if trial % 7 == 0:          # self-loop heavy
            d = s.copy()
        if trial % 11 == 0:         # extreme addresses
            s[: n // 2] = 0xFFFFFFFF
        np.testing.assert_array_equal(one(s, d), brute_force(s, d), err_msg=f"trial {trial}")
        checked += 1
    assert checked == 3000


def test_oracle_vs_brute_force_batched():
    rng = np.random.default_rng(99)
    sizes = rng.integers(0, 60, 40)
    off = synth.offsets_from_sizes(sizes)
    s = rng.integers(0, 6, off[-1]).astype(np.uint32)
    d = rng.integers(0, 6, off[-1]).astype(np.uint32)
    got = oracle.window_stats(s, d, off, threads=4)
    for w in range(40):
        np.testing.assert_array_equal(got[w], brute_force(s[off[w]:off[w + 1]], d[off[w]:off[w + 1]]))


@pytest.mark.parametrize("maker", ["uniform_single", "zipf_batch", "skewed_large",
                                   "uneven_batch", "serving_stream"])
def test_oracle_vs_numpy_unique_medium(maker):
    fn = synth.WORKLOADS[maker]
    if maker in ("uneven_batch", "serving_stream"):
        wl = fn(seed=5, num_windows=3, lo_log2=8, hi_log2=15)
    else:
        wl = fn(seed=5, num_windows=2, log2_window=15)
    src, dst = wl.generate()
    got = oracle.window_stats(src, dst, wl.offsets, threads=2)
    for w in range(wl.num_windows):
        a, b = int(wl.offsets[w]), int(wl.offsets[w + 1])
        np.testing.assert_array_equal(got[w], numpy_unique(src[a:b], dst[a:b]), err_msg=f"w{w}")
        check_invariants(got[w], b - a)


def test_entities_match_numpy_unique():
    src, dst, off = _small_workload(21, windows=1)
    e = oracle.window_entities(src, dst)
    keys = (src.astype(np.uint64) << np.uint64(32)) | dst.astype(np.uint64)
    uk, cnt = np.unique(keys, return_counts=True)
    np.testing.assert_array_equal(e["link_keys"], uk)
    np.testing.assert_array_equal(e["link_counts"], cnt.astype(np.uint64))
    us, cs = np.unique(src, return_counts=True)
    np.testing.assert_array_equal(e["row_ids"], us)
    np.testing.assert_array_equal(e["row_packets"], cs.astype(np.uint64))
    ud, cd = np.unique(dst, return_counts=True)
    np.testing.assert_array_equal(e["col_ids"], ud)
    np.testing.assert_array_equal(e["col_packets"], cd.astype(np.uint64))
    # fan-out / fan-in: distinct links per source / destination
    _, fo = np.unique(uk >> np.uint64(32), return_counts=True)
    _, fi = np.unique(uk & np.uint64(0xFFFFFFFF), return_counts=True)
    np.testing.assert_array_equal(e["row_links"], fo.astype(np.uint64))
    np.testing.assert_array_equal(e["col_links"], fi.astype(np.uint64))


def test_uniform_window_statistical_sanity():
    # not a parity pin: a uniform window over M = 4096^2 possible pairs has
    # E[nnz] = M (1 - exp(-n/M)); the observed value must be close.
    wl = synth.uniform_single(seed=1)
    src, dst = wl.generate()
    st = oracle.window_stats(src, dst, wl.offsets)[0]
    n, M = 1 << 17, 4096.0 ** 2
    expected = M * (1 - np.exp(-n / M))
    assert abs(int(st[1]) - expected) < 200
    assert int(st[3]) == 4096 and int(st[6]) == 4096
