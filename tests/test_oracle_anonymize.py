"""Pins for the oracle's address anonymization (Section IV, "IP Address
Anonymization").

The paper lists the unique source and destination addresses, shuffles the
sequence 0..N-1 and maps the i-th unique address to the i-th shuffled value.
The oracle lists the unique addresses in ascending order and uses a seeded
pseudo-random permutation (a four-round Feistel network with cycle walking)
for the shuffle.  Pinned here:

* the unique list equals numpy.union1d (values and order) and its length the
  globally unique IP count of the statistics oracle;
* the permutation is a bijection of [0, N) for every N tried (exhaustively),
  changes with the seed, and its values look uniform (a loose chi-square on
  where 0 lands over many seeds -- a sanity check, not parity);
* the anonymized columns are pi(rank) with rank the position in the unique
  list, the same address gets the same value in both columns, every value is
  below N, and the nine statistics of every window are unchanged by the
  anonymization (an injective relabelling of addresses, the metamorphic
  relation the statistics must satisfy);
* planted mistakes in copies of the oracle (a lost column, two maps for the
  two columns, a permutation that is not one) fail these pins.

The permutation's individual values are fixed only by its written definition
(there are no published values to compare with): parity unpinned beyond the
properties above.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from conftest import ROOT


@pytest.mark.parametrize("n", list(range(0, 70)) + [255, 256, 257, 1000, 4095, 4096, 5000])
def test_permutation_is_a_bijection(n):
    for seed in (0, 1, 0xDEADBEEF12345678):
        vals = [oracle.permute(i, n, seed) for i in range(n)]
        assert sorted(vals) == list(range(n)), (n, seed)


def test_permutation_depends_on_the_seed_and_looks_uniform():
    n = 1000
    a = [oracle.permute(i, n, 1) for i in range(n)]
    b = [oracle.permute(i, n, 2) for i in range(n)]
    assert a != b
    assert sum(x == i for i, x in enumerate(a)) < 10          # few fixed points
    # where 0 lands over 4000 seeds: 10 bins of 100 values, expected 400 each
    counts = np.bincount([oracle.permute(0, n, s) // 100 for s in range(4000)], minlength=10)
    chi2 = float(((counts - 400.0) ** 2 / 400.0).sum())
    assert chi2 < 40.0, counts


def test_unique_list_is_sorted_union():
    wl = synth.zipf_batch(seed=3, num_windows=2, log2_window=12)
    src, dst = wl.generate()
    u = oracle.unique_addresses(src, dst)
    np.testing.assert_array_equal(u, np.union1d(src, dst))
    assert u.size == int(oracle.unique_ips(src, dst, np.array([0, src.size], np.int64))[0])


def test_mapping_is_pi_of_rank_and_consistent_across_columns():
    rng = np.random.default_rng(4)
    src = rng.integers(0, 50, 3000).astype(np.uint32)
    dst = rng.integers(25, 90, 3000).astype(np.uint32)
    a, b, n = oracle.anonymize(src, dst, seed=77)
    u = oracle.unique_addresses(src, dst)
    assert n == u.size
    pi = np.array([oracle.permute(i, n, 77) for i in range(n)], np.uint32)
    np.testing.assert_array_equal(a, pi[np.searchsorted(u, src)])
    np.testing.assert_array_equal(b, pi[np.searchsorted(u, dst)])
    assert a.max() < n and b.max() < n
    both = np.intersect1d(src, dst)
    for x in both[:10]:
        assert len(set(a[src == x]) | set(b[dst == x])) == 1


def test_statistics_survive_anonymization():
    for maker in ("zipf_batch", "skewed_large", "uniform_single"):
        wl = synth.WORKLOADS[maker](seed=2, num_windows=3 if maker != "uniform_single" else 1,
                                    log2_window=13)
        src, dst = wl.generate()
        a, b, _ = oracle.anonymize(src, dst, seed=5)
        np.testing.assert_array_equal(oracle.window_stats(a, b, wl.offsets),
                                      oracle.window_stats(src, dst, wl.offsets))


def test_empty_and_single_address():
    a, b, n = oracle.anonymize(np.zeros(0, np.uint32), np.zeros(0, np.uint32), 1)
    assert n == 0 and a.size == 0
    a, b, n = oracle.anonymize(np.full(5, 7, np.uint32), np.full(5, 7, np.uint32), 1)
    assert n == 1 and (a == 0).all() and (b == 0).all()


MUTANTS = {
    "destinations_not_listed": ("    ips.insert(dst[i]);\n  }\n  const uint64_t N = ips.size();",
                                "  }\n  const uint64_t N = ips.size();"),
    "second_map_for_destinations": ("    adst[i] = static_cast<uint32_t>(id[dst[i]]);",
                                    "    adst[i] = static_cast<uint32_t>(permute(id[dst[i]], N, seed));"),
    "not_a_permutation": ("  while (y >= N) y = feistel(y, b / 2, seed);\n  return y;",
                          "  return y % N;"),
}


def _anonymize_with(tmp_path, name, text, src, dst):
    cpp = tmp_path / f"{name}.cpp"
    so = tmp_path / f"lib{name}.so"
    cpp.write_text(text)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread",
                           str(cpp), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    lib.nsgc_oracle_anonymize.restype = ctypes.c_int
    lib.nsgc_oracle_anonymize.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p]
    a = np.zeros(src.size, np.uint32)
    b = np.zeros(src.size, np.uint32)
    n = np.zeros(1, np.uint64)
    assert lib.nsgc_oracle_anonymize(src.ctypes.data, dst.ctypes.data, src.size, 9,
                                     a.ctypes.data, b.ctypes.data, n.ctypes.data) == 0
    return a, b, int(n[0])


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    with open(os.path.join(ROOT, "oracle", "nsgc_oracle.cpp")) as fh:
        text = fh.read()
    assert text.count(old) == 1, name
    rng = np.random.default_rng(10)
    src = rng.integers(0, 300, 5000).astype(np.uint32)
    dst = rng.integers(150, 600, 5000).astype(np.uint32)
    off = np.array([0, 2500, 5000], np.int64)
    a, b, n = _anonymize_with(tmp_path, name, text.replace(old, new), src, dst)
    caught = (n != np.union1d(src, dst).size or a.max(initial=0) >= max(n, 1)
              or b.max(initial=0) >= max(n, 1)
              or not np.array_equal(oracle.window_stats(a, b, off),
                                    oracle.window_stats(src, dst, off))
              or np.unique(np.concatenate([a, b])).size != np.union1d(src, dst).size)
    assert caught
