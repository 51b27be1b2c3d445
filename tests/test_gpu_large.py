"""GPU parity of the large-window tier (one window at a time, by sorting).

With the tier's threshold lowered to its minimum (2^20 packets) it is
compared bit for bit with the oracle on windows of every kind: heavy-tailed,
skewed with a super-source and a super-destination, tiny alphabets (long
runs of one link), a bijection (no repeats), addresses whose hashed form is
all ones, and batches that mix it with the other tiers, in the batched,
plain, fixed-scratch and timed forms.  At the default threshold it takes a single window of 2^26
packets, compared in full with the oracle, and a single window of 2^30
packets (the whole capture of the paper as one window), checked by the exact
invariants and the src/dst swap (Table III caption: the reverse queries swap
the roles of the two columns).
"""
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_same, gpu_stats, say, to_gpu
from hashed_addresses import DESTINATION_MARKER, SOURCE_MARKER
from test_gpu_fullsize import invariants

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _default_tuning():
    import paper_2509_03653_amd as nsgc
    nsgc.set_tune(nsgc.default_tune())
    yield
    nsgc.set_tune(nsgc.default_tune())


def _threshold(log2):
    import paper_2509_03653_amd as nsgc
    t = nsgc.default_tune()
    t.large_min_log2 = log2
    nsgc.set_tune(t)


def test_large_tier_every_kind_of_window():
    import paper_2509_03653_amd as nsgc
    _threshold(20)
    n = 1 << 20
    rng = np.random.default_rng(3)
    cases = {}
    wl = synth.zipf_batch(seed=2, num_windows=1, log2_window=20)
    cases["zipf"] = wl.generate()
    wl = synth.skewed_large(seed=2, num_windows=1, log2_window=20)
    cases["skewed"] = wl.generate()
    cases["tiny_alphabet"] = (rng.integers(0, 3, n).astype(np.uint32),
                              rng.integers(0, 2, n).astype(np.uint32))
    perm = rng.permutation(n).astype(np.uint32)
    cases["bijection"] = (np.arange(n, dtype=np.uint32), perm)
    s = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    d = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    s[::7] = SOURCE_MARKER
    d[::5] = DESTINATION_MARKER
    s[::11] = 0xFFFFFFFF
    cases["markers"] = (s, d)
    cases["identical"] = (np.full(n, 9, np.uint32), np.full(n, 4, np.uint32))
    off = np.array([0, n], np.int64)
    for name, (src, dst) in cases.items():
        p = nsgc.plan_inspect(off)
        assert int(p["tier"][0]) == 3
        want = oracle.window_stats(src, dst, off)
        for form in ("batched", "plain", "noalloc"):
            say(f"[gpu] large tier {name} {form}")
            assert_same(gpu_stats(src, dst, off, form), want, f"large {name} {form}")


def test_large_tier_mixed_with_other_tiers_and_timed():
    import torch

    import paper_2509_03653_amd as nsgc
    _threshold(20)
    sizes = [(1 << 20) + 3, 5000, 0, 700, (1 << 21) - 1, 300000, 1 << 20]
    off = synth.offsets_from_sizes(sizes)
    wl = synth.zipf_batch(seed=6, num_windows=1, log2_window=4)
    src, dst = synth.fill(off, 21, wl.src_dist, wl.dst_dist)
    tiers = list(nsgc.plan_inspect(off)["tier"])
    assert tiers == [3, 2, 0, 1, 3, 2, 3]
    want = oracle.window_stats(src, dst, off, threads=8)
    for form in ("batched", "plain"):
        say(f"[gpu] mixed tiers {form}")
        assert_same(gpu_stats(src, dst, off, form), want, f"mixed tiers {form}")
    s, d = to_gpu(src), to_gpu(dst)
    out, ph = nsgc.window_stats_timed(s, d, off)
    torch.cuda.synchronize()
    assert_same(out.cpu().numpy().view(np.uint64), want, "mixed tiers timed")
    assert ph["large"] > 0
    # the graph form has no large tier: the same windows go through partitioning
    say("[gpu] mixed tiers graph")
    assert_same(gpu_stats(src, dst, off, "graph"), want, "mixed tiers graph")


def _skewed_window(log2, seed):
    wl = synth.skewed_large(seed=seed, num_windows=1, log2_window=log2)
    say(f"[cpu] generating one skewed window of 2^{log2} packets")
    return wl.generate()


def test_single_window_2e26_exact():
    import paper_2509_03653_amd as nsgc
    src, dst = _skewed_window(26, 7)
    off = np.array([0, src.size], np.int64)
    assert int(nsgc.plan_inspect(off)["tier"][0]) == 3
    got = gpu_stats(src, dst, off)
    say("[cpu] oracle on the 2^26-packet window")
    want = oracle.window_stats(src, dst, off)
    assert_same(got, want, "one window of 2^26 packets")


def test_single_window_2e30_invariants_and_swap():
    import torch

    import paper_2509_03653_amd as nsgc
    src, dst = _skewed_window(30, 8)
    n = src.size
    off = np.array([0, n], np.int64)
    assert int(nsgc.plan_inspect(off)["tier"][0]) == 3
    say(f"[gpu] upload {n} packets")
    s, d = to_gpu(src), to_gpu(dst)
    del src, dst
    out = nsgc.window_stats(s, d, off)          # first call sizes the workspace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = nsgc.window_stats(s, d, off)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    fwd = out.cpu().numpy().view(np.uint64).copy()
    rev = nsgc.window_stats(d, s, off)
    torch.cuda.synchronize()
    rev = rev.cpu().numpy().view(np.uint64).copy()
    say(f"[gpu] one window of 2^30 packets: {ms:.1f} ms; stats {fwd[0].tolist()}")
    invariants(fwd, [n])
    invariants(rev, [n])
    np.testing.assert_array_equal(rev[0], fwd[0][[0, 1, 2, 6, 7, 8, 3, 4, 5]])
    del s, d
    torch.cuda.empty_cache()
    nsgc.release()


def test_single_source_2e28_star():
    # every packet from one source to a distinct destination: a star whose
    # statistics are known in closed form, and its reverse
    import torch

    import paper_2509_03653_amd as nsgc
    n = 1 << 28
    src = np.full(n, 0x0A000001, np.uint32)
    dst = np.arange(n, dtype=np.uint32)
    off = np.array([0, n], np.int64)
    assert int(nsgc.plan_inspect(off)["tier"][0]) == 3
    say(f"[gpu] star of {n} distinct links")
    s, d = to_gpu(src), to_gpu(dst)
    del src, dst
    out = nsgc.window_stats(s, d, off)
    rev = nsgc.window_stats(d, s, off)
    torch.cuda.synchronize()
    want = np.array([[n, n, 1, 1, n, n, n, 1, 1]], np.uint64)
    assert_same(out.cpu().numpy().view(np.uint64), want, "one-source window")
    assert_same(rev.cpu().numpy().view(np.uint64), want[:, [0, 1, 2, 6, 7, 8, 3, 4, 5]],
                "one-destination window")
    del s, d, out, rev
    torch.cuda.empty_cache()
    nsgc.release()
