"""CPU oracle for the per-window traffic-matrix statistics -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the bench's CPU-baseline leg
may import this package.  The product path (``paper_2509_03653_amd``) never
does, and shares no code with it.

The oracle is ``nsgc_oracle.cpp``: an ordered-map implementation of the
definitions in the paper's Table III (valid packets, unique links, max link
packets, unique sources, max source packets, max source fan-out) and of their
reverses obtained by swapping src and dst (Table III caption).  Pins that tie
it to something other than itself live in ``tests/test_oracle_pins.py``:
hand-worked windows (``tests/golden/``), closed forms, invariants,
metamorphic relations, an O(n^2) brute force and a ``numpy.unique``
formulation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libnsgc_oracle.so")
_SRC_PATH = os.path.join(_HERE, "nsgc_oracle.cpp")
_lib = None

STAT_NAMES = (
    "valid_packets",
    "unique_links",
    "max_link_packets",
    "unique_sources",
    "max_source_packets",
    "max_source_fanout",
    "unique_destinations",
    "max_destination_packets",
    "max_destination_fanin",
)


def build_library(force: bool = True) -> str:
    """Compile the oracle with g++ (plain -O2, no tuning)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", _SRC_PATH,
             "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_library(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.nsgc_oracle_window_stats.restype = ctypes.c_int
        lib.nsgc_oracle_window_stats.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_int]
        lib.nsgc_oracle_unique_ips.restype = ctypes.c_int
        lib.nsgc_oracle_unique_ips.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_int]
        lib.nsgc_oracle_permute.restype = ctypes.c_uint64
        lib.nsgc_oracle_permute.argtypes = [ctypes.c_uint64] * 3
        lib.nsgc_oracle_unique_addresses.restype = ctypes.c_int64
        lib.nsgc_oracle_unique_addresses.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                                     ctypes.c_int64, ctypes.c_void_p]
        lib.nsgc_oracle_anonymize.restype = ctypes.c_int
        lib.nsgc_oracle_anonymize.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                              ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]
        lib.nsgc_oracle_window_entities.restype = ctypes.c_int
        lib.nsgc_oracle_window_entities.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64] + [
            ctypes.c_void_p] * 11
        _lib = lib
    return _lib


def window_stats(src, dst, offsets, threads: int = 1) -> np.ndarray:
    """Nine statistics per window, as a (W, 9) uint64 array.

    ``src``/``dst`` are uint32 arrays, ``offsets`` has W+1 non-decreasing
    entries; window w is packets ``[offsets[w], offsets[w+1])``.
    """
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    w = len(offsets) - 1
    out = np.zeros((max(w, 0), 9), dtype=np.uint64)
    if w <= 0:
        return out
    if offsets[-1] > src.size or offsets[-1] > dst.size:
        raise ValueError("offsets run past the packet arrays")
    rc = lib.nsgc_oracle_window_stats(src.ctypes.data, dst.ctypes.data,
                                      offsets.ctypes.data, w, out.ctypes.data,
                                      int(threads))
    if rc != 0:
        raise ValueError("oracle rejected its arguments (offsets must be >= 0 and "
                         "non-decreasing)")
    return out


def unique_ips(src, dst, offsets, threads: int = 1) -> np.ndarray:
    """Globally unique IP addresses per window, |{src} U {dst}| (Section IV,
    "Graph Analytics" paragraph), as a (W,) uint64 array."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    w = len(offsets) - 1
    out = np.zeros(max(w, 0), dtype=np.uint64)
    if w <= 0:
        return out
    if offsets[-1] > src.size or offsets[-1] > dst.size:
        raise ValueError("offsets run past the packet arrays")
    rc = lib.nsgc_oracle_unique_ips(src.ctypes.data, dst.ctypes.data, offsets.ctypes.data, w,
                                    out.ctypes.data, int(threads))
    if rc != 0:
        raise ValueError("oracle rejected its arguments (offsets must be >= 0 and "
                         "non-decreasing)")
    return out


def permute(i: int, n: int, seed: int) -> int:
    """pi(i) of the anonymization's seeded permutation of [0, n)."""
    return int(_load().nsgc_oracle_permute(int(i), int(n), int(seed) & (2 ** 64 - 1)))


def unique_addresses(src, dst) -> np.ndarray:
    """The unique addresses of both columns in ascending order."""
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    out = np.zeros(max(2 * src.size, 1), dtype=np.uint32)
    k = _load().nsgc_oracle_unique_addresses(src.ctypes.data, dst.ctypes.data, src.size,
                                             out.ctypes.data)
    return out[:k]


def anonymize(src, dst, seed: int):
    """Anonymized columns (Section IV, "IP Address Anonymization"): each address
    becomes pi(its rank among the unique addresses in ascending order).
    Returns (anon_src, anon_dst, N)."""
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    if src.size != dst.size:
        raise ValueError("src and dst differ in length")
    a = np.zeros(src.size, np.uint32)
    b = np.zeros(src.size, np.uint32)
    n = np.zeros(1, np.uint64)
    rc = _load().nsgc_oracle_anonymize(src.ctypes.data, dst.ctypes.data, src.size,
                                       int(seed) & (2 ** 64 - 1), a.ctypes.data, b.ctypes.data,
                                       n.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return a, b, int(n[0])


def window_entities(src, dst, begin: int = 0, end: int | None = None) -> dict:
    """Sorted per-entity vectors of one window: A as (key, count), the rows
    (s, r(s), f(s)), the columns (d, c(d), g(d)) and the number of globally
    unique IP addresses |{s} U {d}|."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    if end is None:
        end = src.size
    n = max(end - begin, 1)
    lk = np.zeros(n, np.uint64); lc = np.zeros(n, np.uint64)
    ri = np.zeros(n, np.uint32); rp = np.zeros(n, np.uint64); rl = np.zeros(n, np.uint64)
    ci = np.zeros(n, np.uint32); cp = np.zeros(n, np.uint64); cl = np.zeros(n, np.uint64)
    nl = np.zeros(1, np.int64); nr = np.zeros(1, np.int64); nc = np.zeros(1, np.int64)
    rc = lib.nsgc_oracle_window_entities(
        src.ctypes.data, dst.ctypes.data, int(begin), int(end), lk.ctypes.data,
        lc.ctypes.data, nl.ctypes.data, ri.ctypes.data, rp.ctypes.data, rl.ctypes.data,
        nr.ctypes.data, ci.ctypes.data, cp.ctypes.data, cl.ctypes.data, nc.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    a, b, c = int(nl[0]), int(nr[0]), int(nc[0])
    return {
        "link_keys": lk[:a], "link_counts": lc[:a],
        "row_ids": ri[:b], "row_packets": rp[:b], "row_links": rl[:b],
        "col_ids": ci[:c], "col_packets": cp[:c], "col_links": cl[:c],
        "unique_ips": int(unique_ips(src[begin:end], dst[begin:end],
                                     np.array([0, end - begin], np.int64))[0]),
    }
