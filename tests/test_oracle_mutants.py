"""The pins catch plausible slips in the oracle.

Each case copies the oracle's source, plants one mistake (a swapped view, a
dropped term, fan-out counted as packets, a wrong key, a lost packet), builds
the copy with g++ on the CPU, and checks that the golden windows, the closed
forms or the brute force reject it.  The real oracle passes the same checks.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from conftest import ROOT, load_golden_windows
from independent_refs import brute_force

SRC = os.path.join(ROOT, "oracle", "nsgc_oracle.cpp")

MUTANTS = {
    "fanout_counts_packets": ("rows[s].links += 1;", "rows[s].links += a;"),
    "fanin_counts_packets": ("cols[d].links += 1;", "cols[d].links += a;"),
    "column_sum_counts_links": ("cols[d].packets += a;", "cols[d].packets += 1;"),
    "max_link_dropped": ("max_link = std::max(max_link, a);", "max_link = a;"),
    "views_swapped": ("out[3] = static_cast<uint64_t>(rows.size());",
                      "out[3] = static_cast<uint64_t>(cols.size());"),
    "key_ignores_dst": ("A[std::make_pair(src[i], dst[i])] += 1;\n\n  std::map<uint32_t, Totals> rows;",
                        "A[std::make_pair(src[i], src[i])] += 1;\n\n  std::map<uint32_t, Totals> rows;"),
    "last_packet_lost": ("for (int64_t i = begin; i < end; ++i) A[std::make_pair(src[i], dst[i])] += 1;\n\n  std::map<uint32_t, Totals> rows;",
                         "for (int64_t i = begin; i + 1 < end; ++i) A[std::make_pair(src[i], dst[i])] += 1;\n\n  std::map<uint32_t, Totals> rows;"),
    "fanin_max_of_packets": ("max_g = std::max(max_g, e.second.links);",
                             "max_g = std::max(max_g, e.second.packets);"),
    "unique_links_counts_rows": ("out[1] = static_cast<uint64_t>(A.size());",
                                 "out[1] = static_cast<uint64_t>(rows.size());"),
}


def _build(tmp_path, name, text):
    cpp = tmp_path / f"{name}.cpp"
    so = tmp_path / f"lib{name}.so"
    cpp.write_text(text)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread",
                           str(cpp), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    lib.nsgc_oracle_window_stats.restype = ctypes.c_int
    lib.nsgc_oracle_window_stats.argtypes = [ctypes.c_void_p] * 3 + [
        ctypes.c_int64, ctypes.c_void_p, ctypes.c_int]
    return lib


def _stats(lib, src, dst):
    src = np.ascontiguousarray(src, np.uint32)
    dst = np.ascontiguousarray(dst, np.uint32)
    off = np.array([0, src.size], np.int64)
    out = np.zeros(9, np.uint64)
    assert lib.nsgc_oracle_window_stats(src.ctypes.data, dst.ctypes.data, off.ctypes.data,
                                        1, out.ctypes.data, 1) == 0
    return out


def _pins_pass(lib) -> bool:
    for s, d, e in load_golden_windows().values():
        if not np.array_equal(_stats(lib, s, d), e):
            return False
    k, m, t = 4, 6, 3
    ss, dd = np.meshgrid(np.arange(k) + 100, np.arange(m) + 1000, indexing="ij")
    s = np.repeat(ss.ravel(), t)
    d = np.repeat(dd.ravel(), t)
    if not np.array_equal(_stats(lib, s, d), [t * k * m, k * m, t, k, t * m, m, m, t * k, k]):
        return False
    rng = np.random.default_rng(5)
    for _ in range(200):
        n = int(rng.integers(1, 64))
        s = rng.integers(0, 5, n).astype(np.uint32)
        d = rng.integers(0, 5, n).astype(np.uint32)
        if not np.array_equal(_stats(lib, s, d), brute_force(s, d)):
            return False
    return True


def test_unmodified_oracle_passes(tmp_path):
    with open(SRC) as fh:
        assert _pins_pass(_build(tmp_path, "orig", fh.read()))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    with open(SRC) as fh:
        text = fh.read()
    assert text.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    assert not _pins_pass(_build(tmp_path, name, text.replace(old, new)))
