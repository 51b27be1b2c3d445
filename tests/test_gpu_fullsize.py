"""GPU parity at the workloads' full sizes, in the benchmark's launch
configuration (the captured-graph batched form).

  * 1 window of 2^17, uniform over 4096 addresses: every statistic vs the oracle.
  * 64 windows of 2^17 (the benchmark batch): every window vs the oracle.
  * 128 windows of 2^23 with a super-source and a super-destination (2^30
    packets): every window vs the oracle (one window per host thread).
  * 4096 windows log-uniform in [2^10, 2^23] (~3.8e9 packets): every window
    of at least 2^22 packets and a random 5% of the others vs the oracle,
    exact invariants on every window.

The invariants hold for any exact result and are checked on all windows:
stat0 = n; max(stat3, stat6) <= stat1 <= min(n, stat3 * stat6);
stat2 <= min(stat4, stat7); stat5 <= min(stat4, stat6); stat8 <= min(stat7,
stat3); stat3 * stat4 >= n and stat6 * stat7 >= n; every statistic >= 1 for a
non-empty window (all zero for an empty one).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_same, say, to_gpu

pytestmark = pytest.mark.gpu


def invariants(stats, sizes):
    s = np.asarray(stats, dtype=np.uint64).astype(object)   # exact products
    n = np.asarray(sizes, dtype=np.int64)
    bad = []
    for w in range(len(n)):
        x = [int(v) for v in s[w]]
        nw = int(n[w])
        if nw == 0:
            ok = all(v == 0 for v in x)
        else:
            ok = (x[0] == nw and max(x[3], x[6]) <= x[1] <= min(nw, x[3] * x[6])
                  and x[2] <= min(x[4], x[7]) and x[5] <= min(x[4], x[6])
                  and x[8] <= min(x[7], x[3]) and x[3] * x[4] >= nw and x[6] * x[7] >= nw
                  and min(x) >= 1)
        if not ok:
            bad.append((w, x, nw))
    assert not bad, f"{len(bad)} windows break the invariants, first {bad[0]}"


def graph_stats(src, dst, off):
    import torch

    import paper_2509_03653_amd as nsgc
    say(f"[gpu] upload {int(off[-1])} packets")
    s, d = to_gpu(src), to_gpu(dst)
    g = nsgc.Graph(int(off[-1] - off[0]), len(off) - 1)
    try:
        say(f"[gpu] graph launch over {len(off) - 1} windows")
        out = g.launch(s, d, off)
        torch.cuda.synchronize()
        say("[gpu] launch done")
        res = out.cpu().numpy().view(np.uint64).copy()
    finally:
        g.close()
        del s, d
        torch.cuda.empty_cache()
    nsgc.check_valid(res)
    return res


def sampled_oracle(src, dst, off, windows):
    """The oracle on the sampled windows, gathered into one batch so that it
    runs them in parallel (one window per thread)."""
    say(f"[cpu] oracle on windows {list(windows)}")
    parts = [(int(off[w]), int(off[w + 1])) for w in windows]
    s = np.concatenate([src[a:b] for a, b in parts])
    d = np.concatenate([dst[a:b] for a, b in parts])
    o = synth.offsets_from_sizes([b - a for a, b in parts])
    return oracle.window_stats(s, d, o, threads=min(len(parts), _host_threads()))


def test_uniform_single_window_full():
    wl = synth.uniform_single(seed=1)
    src, dst = wl.generate()
    got = graph_stats(src, dst, wl.offsets)
    want = oracle.window_stats(src, dst, wl.offsets)
    assert_same(got, want, "uniform 2^17")
    # the pool has 4096 addresses: every one appears as a source and a destination
    assert int(got[0, 3]) == 4096 and int(got[0, 6]) == 4096


def test_benchmark_batch_full():
    wl = synth.zipf_batch(seed=1)
    src, dst = wl.generate()
    got = graph_stats(src, dst, wl.offsets)
    say("[cpu] oracle on the whole batch")
    want = oracle.window_stats(src, dst, wl.offsets, threads=16)
    assert_same(got, want, "64 x 2^17")


def _host_threads():
    import os
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return 8


def test_skewed_2e30_packets_every_window():
    wl = synth.skewed_large(seed=1)
    say("[cpu] generating 128 x 2^23 packets")
    src, dst = wl.generate()
    got = graph_stats(src, dst, wl.offsets)
    invariants(got, np.diff(wl.offsets))
    say("[cpu] oracle on all 128 windows")
    want = oracle.window_stats(src, dst, wl.offsets, threads=_host_threads())
    assert_same(got, want, "skewed 128 x 2^23")
    # the super-source (10% of packets) dominates the row maxima
    assert np.all(got[:, 4] >= (1 << 23) // 20)


def test_uneven_4096_windows_large_ones_and_a_sample():
    wl = synth.uneven_batch(seed=1)
    say(f"[cpu] generating {wl.num_packets} packets in 4096 windows")
    src, dst = wl.generate()
    sizes = np.diff(wl.offsets)
    got = graph_stats(src, dst, wl.offsets)
    invariants(got, sizes)
    rng = np.random.default_rng(7)
    big = np.flatnonzero(sizes >= (1 << 22))
    small = np.flatnonzero(sizes < (1 << 22))
    sample = sorted(set(big.tolist()) | set(rng.choice(small, len(small) // 20, replace=False).tolist())
                    | {int(np.argmin(sizes))})
    say(f"[cpu] oracle on {len(sample)} windows ({len(big)} of at least 2^22 packets)")
    want = sampled_oracle(src, dst, wl.offsets, sample)
    assert_same(got[sample], want, "uneven: large windows and a 5% sample")
