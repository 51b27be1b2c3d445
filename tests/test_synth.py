"""The seeded generators: determinism and the distributions they claim."""
import numpy as np
import pytest

import synth


def test_deterministic_and_thread_independent():
    wl = synth.zipf_batch(seed=3, num_windows=5, log2_window=17)
    a = wl.generate(threads=1)
    b = wl.generate(threads=7)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    c = synth.zipf_batch(seed=4, num_windows=5, log2_window=17).generate()
    assert not np.array_equal(a[0], c[0])


def test_window_independent_of_batch():
    wl = synth.uneven_batch(seed=2, num_windows=20, lo_log2=8, hi_log2=17)
    src, dst = wl.generate()
    s2, d2, off2 = wl.generate_windows([3, 17, 5])
    for i, w in enumerate([3, 17, 5]):
        np.testing.assert_array_equal(s2[off2[i]:off2[i + 1]], src[wl.offsets[w]:wl.offsets[w + 1]])
        np.testing.assert_array_equal(d2[off2[i]:off2[i + 1]], dst[wl.offsets[w]:wl.offsets[w + 1]])


def test_pool_is_a_bijection():
    ranks = np.arange(1 << 20, dtype=np.uint64)
    addr = np.array([synth.pool_address(int(r), 0xABCDEF) for r in ranks[:5000]])
    assert np.unique(addr).size == 5000


def test_uniform_pool_of_4096():
    wl = synth.uniform_single(seed=1)
    src, dst = wl.generate()
    assert src.size == 1 << 17
    assert np.unique(src).size == 4096 and np.unique(dst).size == 4096
    counts = np.unique(src, return_counts=True)[1]
    assert abs(counts.mean() - 32.0) < 1e-9 and counts.max() < 80


@pytest.mark.parametrize("alpha,n", [(1.0, 1 << 24), (1.2, 1 << 20), (1.3, 1 << 26), (0.8, 1000)])
def test_zipf_matches_truncated_law(alpha, n):
    draws = 400_000
    r = synth.zipf_ranks(draws, 17, alpha, n)
    assert r.min() >= 1 and r.max() <= n
    k = np.arange(1, min(n, 1 << 22) + 1, dtype=np.float64)
    norm = np.sum(k ** -alpha)
    if n > k.size:   # tail of the normaliser by the integral approximation
        a, b = k.size + 0.5, n + 0.5
        norm += (b ** (1 - alpha) - a ** (1 - alpha)) / (1 - alpha) if alpha != 1 else np.log(b / a)
    for rank in (1, 2, 3, 10):
        p = rank ** -alpha / norm
        obs = np.count_nonzero(r == rank) / draws
        sd = np.sqrt(p * (1 - p) / draws)
        assert abs(obs - p) < 5 * sd + 1e-4, (rank, obs, p)


def test_super_addresses_outside_pool():
    wl = synth.skewed_large(seed=1, num_windows=1, log2_window=16)
    src, dst = wl.generate()
    s_star = synth.pool_address(1 << 26, synth.POOL_KEY_C)
    d_star = synth.pool_address((1 << 26) + 1, synth.POOL_KEY_C)
    fs = np.count_nonzero(src == s_star) / src.size
    fd = np.count_nonzero(dst == d_star) / dst.size
    assert abs(fs - 0.10) < 0.01 and abs(fd - 0.01) < 0.003
    pool = {synth.pool_address(i, synth.POOL_KEY_C) for i in range(1000)}
    assert s_star not in pool and d_star not in pool


def test_log_uniform_sizes():
    s = synth.log_uniform_sizes(20000, 1, 10, 23)
    assert s.min() >= 1 << 10 and s.max() <= 1 << 23
    lg = np.log2(s.astype(np.float64))
    assert abs(lg.mean() - 16.5) < 0.1
    s2 = synth.log_uniform_sizes(20000, 1, 10, 23)
    np.testing.assert_array_equal(s, s2)


def test_exponential_gaps_mean():
    g = synth.exponential_gaps(200000, 1, 2.5)
    assert g.min() >= 0 and abs(g.mean() - 2.5) < 0.03
