"""GPU parity of the address anonymization (nsgc_anonymize) with the oracle,
bit for bit: both anonymized columns and the number of unique addresses, for
empty input, a single address, tiny alphabets with the extreme addresses,
uniform random 32-bit addresses and the 64 x 2^17 Zipf batch; in place as
well.  The anonymized batch keeps every window's nine statistics."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import gpu_stats, say, to_gpu

pytestmark = pytest.mark.gpu


def check(src, dst, seed, what, in_place=False):
    import torch

    import paper_2509_03653_amd as nsgc
    say(f"[gpu] anonymize {what}: {src.size} packets")
    want_s, want_d, want_n = oracle.anonymize(src, dst, seed)
    s, d = to_gpu(src), to_gpu(dst)
    if in_place:
        a, b, num = nsgc.anonymize(s, d, seed, out_src=s, out_dst=d)
    else:
        a, b, num = nsgc.anonymize(s, d, seed)
    torch.cuda.synchronize()
    assert int(num.cpu()[0]) == want_n, what
    np.testing.assert_array_equal(a.cpu().numpy().view(np.uint32), want_s, err_msg=what)
    np.testing.assert_array_equal(b.cpu().numpy().view(np.uint32), want_d, err_msg=what)
    return want_s, want_d


def test_small_cases():
    check(np.zeros(0, np.uint32), np.zeros(0, np.uint32), 1, "empty")
    check(np.full(9, 123, np.uint32), np.full(9, 123, np.uint32), 1, "one address")
    rng = np.random.default_rng(5)
    for trial, alphabet in enumerate((2, 3, 17, 1000)):
        n = int(rng.integers(1, 5000))
        pool = np.array([0, 0xFFFFFFFF, 1, 0x80000000] + list(range(5, 5 + alphabet)), np.uint32)
        s = pool[rng.integers(0, pool.size, n)]
        d = pool[rng.integers(0, pool.size, n)]
        check(s, d, 1000 + trial, f"alphabet {alphabet}")


def test_random_addresses_and_in_place():
    rng = np.random.default_rng(6)
    n = 300000
    s = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    d = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    check(s, d, 0xABCDEF, "uniform random")
    check(s, d, 0xABCDEF, "uniform random, in place", in_place=True)


def test_benchmark_batch_and_statistics_unchanged():
    wl = synth.zipf_batch(seed=1)
    src, dst = wl.generate()
    a, b = check(src, dst, 42, "64 x 2^17 Zipf")
    np.testing.assert_array_equal(gpu_stats(a, b, wl.offsets), gpu_stats(src, dst, wl.offsets))
