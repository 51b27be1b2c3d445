"""Seeded synthetic packet windows (inputs for tests, the bench and the serving loop).

The paper's measurements run on one anonymized capture of 2^30 packets,
distributed as 128 archives x 64 matrices, i.e. windows of 2^17 packets
(Section III "Inputs", Section IV "GraphBLAS format").  That capture is not
available here; the workloads below are seeded heavy-tailed stand-ins with the
same window structure.  This module draws addresses and sizes only: it
contains none of the window-statistics arithmetic, so the HIP path and the CPU
oracle can both consume what it produces.

The generator itself is plain C (``synth.c``), built into ``libsynth.so`` by
``build_library()``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_SRC_PATH = os.path.join(_HERE, "synth.c")
_lib = None

# Pool keys of the rank -> address bijection (one per named pool).
POOL_KEY_A = 0x44303743
POOL_KEY_B = 0x81912ED7
POOL_KEY_C = 0x2C1B3C6D


class _Dist(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("pad0", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("pool_size", ctypes.c_uint64),
        ("pool_key", ctypes.c_uint32),
        ("super_rank", ctypes.c_uint32),
        ("p_super", ctypes.c_double),
    ]


@dataclass(frozen=True)
class AddressDist:
    """Distribution of one address column.

    kind: "uniform" over the pool or "zipf" (truncated, exponent ``alpha``)
    over the pool's popularity ranks.  With probability ``p_super`` a draw is
    replaced by the pool's super address (rank ``super_rank``, outside the
    pool, so it never coincides with a pool address).
    """

    kind: str
    pool_size: int
    pool_key: int
    alpha: float = 1.0
    p_super: float = 0.0
    super_rank: int = 0

    def _c(self) -> _Dist:
        d = _Dist()
        d.kind = {"uniform": 0, "zipf": 1}[self.kind]
        d.alpha = float(self.alpha)
        d.pool_size = int(self.pool_size)
        d.pool_key = int(self.pool_key) & 0xFFFFFFFF
        d.super_rank = int(self.super_rank) & 0xFFFFFFFF
        d.p_super = float(self.p_super)
        return d


def build_library(force: bool = True) -> str:
    """Compile ``synth.c`` into ``libsynth.so`` with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", _SRC_PATH,
             "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_library(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_fill.restype = ctypes.c_int
        lib.synth_fill.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(_Dist),
            ctypes.POINTER(_Dist), ctypes.c_int]
        lib.synth_log_uniform_sizes.restype = None
        lib.synth_log_uniform_sizes.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
            ctypes.c_double]
        lib.synth_exponential_gaps.restype = None
        lib.synth_exponential_gaps.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double]
        lib.synth_uniform.restype = None
        lib.synth_uniform.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64]
        lib.synth_zipf_ranks.restype = None
        lib.synth_zipf_ranks.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
            ctypes.c_uint64]
        lib.synth_pool_address.restype = ctypes.c_uint32
        lib.synth_pool_address.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        _lib = lib
    return _lib


def default_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def fill(offsets, seed: int, src_dist: AddressDist, dst_dist: AddressDist,
         first_window: int = 0, threads: int | None = None, out_src=None, out_dst=None):
    """Draw the packets of windows ``[offsets[w], offsets[w+1])``.

    Returns ``(src, dst)`` as uint32 arrays of length ``offsets[-1]``
    (positions before ``offsets[0]`` are left zero).  Window ``w`` uses the
    random sub-streams of window number ``first_window + w``, so a window's
    packets do not depend on the other windows of the batch.
    """
    lib = _load()
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    w = len(offsets) - 1
    total = int(offsets[-1]) if w >= 0 else 0
    src = out_src if out_src is not None else np.zeros(total, dtype=np.uint32)
    dst = out_dst if out_dst is not None else np.zeros(total, dtype=np.uint32)
    assert src.dtype == np.uint32 and dst.dtype == np.uint32
    assert src.size >= total and dst.size >= total
    sd, dd = src_dist._c(), dst_dist._c()
    rc = lib.synth_fill(src.ctypes.data, dst.ctypes.data, offsets.ctypes.data, w,
                        int(first_window), int(seed) & 0xFFFFFFFFFFFFFFFF,
                        ctypes.byref(sd), ctypes.byref(dd),
                        int(threads or default_threads()))
    if rc != 0:
        raise ValueError("synth_fill rejected its arguments")
    return src, dst


def log_uniform_sizes(count: int, seed: int, lo_log2: float, hi_log2: float) -> np.ndarray:
    out = np.zeros(count, dtype=np.int64)
    _load().synth_log_uniform_sizes(out.ctypes.data, count, seed, lo_log2, hi_log2)
    return out


def exponential_gaps(count: int, seed: int, mean: float) -> np.ndarray:
    out = np.zeros(count, dtype=np.float64)
    _load().synth_exponential_gaps(out.ctypes.data, count, seed, mean)
    return out


def uniform(count: int, seed: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.float64)
    _load().synth_uniform(out.ctypes.data, count, seed)
    return out


def zipf_ranks(count: int, seed: int, alpha: float, n: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    _load().synth_zipf_ranks(out.ctypes.data, count, seed, alpha, n)
    return out


def pool_address(rank: int, key: int) -> int:
    return int(_load().synth_pool_address(rank, key))


def offsets_from_sizes(sizes) -> np.ndarray:
    sizes = np.asarray(sizes, dtype=np.int64)
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


# --------------------------------------------------------------------------
# Named workloads.  Each is described by what it is and its sizes; the
# ``num_windows`` / ``log2_window`` arguments scale a workload down for tests
# while keeping its traffic mix.
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    offsets: np.ndarray
    src_dist: AddressDist
    dst_dist: AddressDist
    seed: int
    description: str
    extra: dict = field(default_factory=dict)

    @property
    def num_windows(self) -> int:
        return len(self.offsets) - 1

    @property
    def num_packets(self) -> int:
        return int(self.offsets[-1])

    def generate(self, threads: int | None = None):
        return fill(self.offsets, self.seed, self.src_dist, self.dst_dist, threads=threads)

    def generate_windows(self, windows, threads: int | None = None):
        """Packets of the selected windows only, as (src, dst, offsets)."""
        windows = list(windows)
        sizes = [int(self.offsets[w + 1] - self.offsets[w]) for w in windows]
        off = offsets_from_sizes(sizes)
        src = np.zeros(int(off[-1]), dtype=np.uint32)
        dst = np.zeros(int(off[-1]), dtype=np.uint32)
        for i, w in enumerate(windows):
            o = np.array([off[i], off[i + 1]], dtype=np.int64)
            fill(o, self.seed, self.src_dist, self.dst_dist, first_window=w,
                 threads=threads, out_src=src, out_dst=dst)
        return src, dst, off


def uniform_single(seed: int = 1, num_windows: int = 1, log2_window: int = 17) -> Workload:
    """One window of 2^17 packets; src and dst i.i.d. uniform over one pool of
    4096 addresses."""
    pool = AddressDist("uniform", 4096, POOL_KEY_A)
    off = offsets_from_sizes([1 << log2_window] * num_windows)
    return Workload("uniform_1x2^17_pool4096", off, pool, pool, seed,
                    "1 window x 2^17 packets, uniform over 4096 addresses")


def zipf_batch(seed: int = 1, num_windows: int = 64, log2_window: int = 17) -> Workload:
    """64 windows of 2^17 packets; src Zipf(1.2) over a pool of 2^20 addresses,
    dst Zipf(1.0) over a separate pool of 2^24 addresses, drawn independently."""
    s = AddressDist("zipf", 1 << 20, POOL_KEY_A, alpha=1.2)
    d = AddressDist("zipf", 1 << 24, POOL_KEY_B, alpha=1.0)
    off = offsets_from_sizes([1 << log2_window] * num_windows)
    return Workload("zipf_64x2^17", off, s, d, seed,
                    "64 windows x 2^17 packets, src Zipf(1.2)/2^20, dst Zipf(1.0)/2^24")


def skewed_large(seed: int = 1, num_windows: int = 128, log2_window: int = 23) -> Workload:
    """128 windows of 2^23 packets; per packet the src is a single super-source
    with probability 0.10 and the dst a single super-destination with
    probability 0.01; otherwise both are Zipf(1.3) over one shared pool of
    2^26 addresses.  The super addresses lie outside the pool."""
    pool_size = 1 << 26
    s = AddressDist("zipf", pool_size, POOL_KEY_C, alpha=1.3, p_super=0.10,
                    super_rank=pool_size)
    d = AddressDist("zipf", pool_size, POOL_KEY_C, alpha=1.3, p_super=0.01,
                    super_rank=pool_size + 1)
    off = offsets_from_sizes([1 << log2_window] * num_windows)
    return Workload("skewed_128x2^23", off, s, d, seed,
                    "128 windows x 2^23 packets, 10% super-source, 1% super-destination, "
                    "Zipf(1.3)/2^26")


def uneven_batch(seed: int = 1, num_windows: int = 4096, lo_log2: float = 10,
                 hi_log2: float = 23) -> Workload:
    """4096 windows with sizes log-uniform in [2^10, 2^23]; src and dst
    Zipf(1.1) over one shared pool of 2^22 addresses, drawn independently."""
    pool = AddressDist("zipf", 1 << 22, POOL_KEY_A, alpha=1.1)
    sizes = log_uniform_sizes(num_windows, seed, lo_log2, hi_log2)
    off = offsets_from_sizes(sizes)
    return Workload("uneven_4096_2^10..2^23", off, pool, pool, seed,
                    "4096 windows, log-uniform sizes in [2^10, 2^23], Zipf(1.1)/2^22")


def serving_stream(seed: int = 1, num_windows: int = 2200, lo_log2: float = 12,
                   hi_log2: float = 22) -> Workload:
    """Arriving windows with sizes log-uniform in [2^12, 2^22]; src and dst
    Zipf(1.2) over one shared pool of 2^24 addresses."""
    pool = AddressDist("zipf", 1 << 24, POOL_KEY_B, alpha=1.2)
    sizes = log_uniform_sizes(num_windows, seed, lo_log2, hi_log2)
    off = offsets_from_sizes(sizes)
    return Workload("serving_2^12..2^22", off, pool, pool, seed,
                    "Poisson-arriving windows, log-uniform sizes in [2^12, 2^22], "
                    "Zipf(1.2)/2^24")


WORKLOADS = {
    "uniform_single": uniform_single,
    "zipf_batch": zipf_batch,
    "skewed_large": skewed_large,
    "uneven_batch": uneven_batch,
    "serving_stream": serving_stream,
}
