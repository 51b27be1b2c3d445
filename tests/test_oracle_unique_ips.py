"""Pins for the oracle's count of globally unique IP addresses per window.

Section IV ("Graph Analytics" paragraph) takes the unique values of each
column and removes the values common to both; the count is |S U D| for the
source set S and destination set D of a window.  Pinned by hand-worked
windows (tests/golden/hand_unique_ips.txt), closed forms, an O(n^2) brute
force, numpy.union1d, the bounds max(|S|, |D|) <= |S U D| <= |S| + |D|, and
metamorphic relations (the src/dst swap and a relabelling applied to both
columns leave it unchanged).  Planted mistakes in copies of the oracle
(only one column counted, the common values counted twice, the last packet
lost) must fail these pins.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from conftest import ROOT, load_golden_windows
from independent_refs import brute_force_unique_ips


def load_golden_ips():
    path = os.path.join(ROOT, "tests", "golden", "hand_unique_ips.txt")
    out = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, value, _ = [p.strip() for p in line.split("|")]
            out[name] = int(value)
    return out


def ips(src, dst):
    src = np.asarray(src, dtype=np.uint32)
    dst = np.asarray(dst, dtype=np.uint32)
    return int(oracle.unique_ips(src, dst, np.array([0, src.size], np.int64))[0])


@pytest.mark.parametrize("name", sorted(load_golden_ips()))
def test_hand_worked(name):
    s, d, _ = load_golden_windows()[name]
    assert ips(s, d) == load_golden_ips()[name]
    assert brute_force_unique_ips(s, d) == load_golden_ips()[name]


@pytest.mark.parametrize("n", [1, 2, 17, 1000])
def test_closed_forms(n):
    a = np.arange(n, dtype=np.uint32)
    assert ips(np.full(n, 7), np.arange(100, 100 + n)) == n + 1      # star
    assert ips(a, a + 5000) == 2 * n                                   # disjoint bijection
    assert ips(a, a) == n                                              # self-loops only
    assert ips(np.full(n, 3), np.full(n, 4)) == 2                      # one repeated link
    assert ips(a, (a + 1) % n) == n                                    # a cycle


def test_brute_force_tiny_windows():
    rng = np.random.default_rng(77)
    for trial in range(1500):
        n = int(rng.integers(0, 80))
        alphabet = int(rng.choice([1, 2, 3, 7, 50, 2 ** 32]))
        s = rng.integers(0, alphabet, n, dtype=np.uint64).astype(np.uint32)
        d = rng.integers(0, alphabet, n, dtype=np.uint64).astype(np.uint32)
        if trial % 9 == 0:
            s[: n // 2] = 0xFFFFFFFF
        assert ips(s, d) == brute_force_unique_ips(s, d), trial


def test_numpy_union_and_bounds_batched():
    wl = synth.zipf_batch(seed=4, num_windows=6, log2_window=13)
    src, dst = wl.generate()
    got = oracle.unique_ips(src, dst, wl.offsets, threads=3)
    st = oracle.window_stats(src, dst, wl.offsets)
    for w in range(wl.num_windows):
        a, b = int(wl.offsets[w]), int(wl.offsets[w + 1])
        assert int(got[w]) == np.union1d(src[a:b], dst[a:b]).size
        assert max(st[w, 3], st[w, 6]) <= got[w] <= st[w, 3] + st[w, 6]


def test_swap_and_common_relabelling():
    rng = np.random.default_rng(8)
    s = rng.integers(0, 300, 4000).astype(np.uint32)
    d = rng.integers(0, 300, 4000).astype(np.uint32)
    base = ips(s, d)
    assert ips(d, s) == base
    perm = rng.permutation(1 << 20).astype(np.uint32)          # injective on [0, 2^20)
    assert ips(perm[s], perm[d]) == base


def test_empty_windows_and_offsets():
    s = np.array([1, 2, 3], np.uint32)
    d = np.array([2, 2, 9], np.uint32)
    got = oracle.unique_ips(s, d, np.array([0, 0, 2, 2, 3], np.int64))
    np.testing.assert_array_equal(got, [0, 2, 0, 2])


MUTANTS = {
    "sources_only": ("  for (int64_t i = begin; i < end; ++i) {\n    ips.insert(src[i]);\n    ips.insert(dst[i]);\n  }",
                     "  for (int64_t i = begin; i < end; ++i) {\n    ips.insert(src[i]);\n  }"),
    "common_counted_twice": ("  std::set<uint32_t> ips;\n  for (int64_t i = begin; i < end; ++i) {\n    ips.insert(src[i]);\n    ips.insert(dst[i]);\n  }\n  return static_cast<uint64_t>(ips.size());",
                             "  std::set<uint32_t> a, b;\n  for (int64_t i = begin; i < end; ++i) {\n    a.insert(src[i]);\n    b.insert(dst[i]);\n  }\n  return static_cast<uint64_t>(a.size() + b.size());"),
    "last_packet_lost": ("  std::set<uint32_t> ips;\n  for (int64_t i = begin; i < end; ++i) {",
                         "  std::set<uint32_t> ips;\n  for (int64_t i = begin; i + 1 < end; ++i) {"),
}


def _mutant_ips(tmp_path, name, text, src, dst):
    cpp = tmp_path / f"{name}.cpp"
    so = tmp_path / f"lib{name}.so"
    cpp.write_text(text)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread",
                           str(cpp), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    lib.nsgc_oracle_unique_ips.restype = ctypes.c_int
    lib.nsgc_oracle_unique_ips.argtypes = [ctypes.c_void_p] * 3 + [
        ctypes.c_int64, ctypes.c_void_p, ctypes.c_int]
    src = np.ascontiguousarray(src, np.uint32)
    dst = np.ascontiguousarray(dst, np.uint32)
    off = np.array([0, src.size], np.int64)
    out = np.zeros(1, np.uint64)
    assert lib.nsgc_oracle_unique_ips(src.ctypes.data, dst.ctypes.data, off.ctypes.data, 1,
                                      out.ctypes.data, 1) == 0
    return int(out[0])


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    with open(os.path.join(ROOT, "oracle", "nsgc_oracle.cpp")) as fh:
        text = fh.read()
    assert text.count(old) == 1, name
    text = text.replace(old, new)
    golden = load_golden_ips()
    caught = any(_mutant_ips(tmp_path, name, text, s, d) != golden[k]
                 for k, (s, d, _) in load_golden_windows().items())
    assert caught
