"""Per-window traffic-matrix statistics on AMD Instinct MI355X (gfx950).

Thin binding over the C ABI of ``libnsgc.so`` (``include/nsgc.h``): argument
marshalling only.  Every step of the computation runs in the library's HIP
kernels; PyTorch supplies device memory and streams.  There is no CPU
fallback: calls fail if the library is not built or the tensors are not on a
GPU.

Statistics per window, in order (arXiv 2509.03653, Table III and its src/dst
reverse): valid packets, unique links, max link packets, unique sources, max
source packets, max source fan-out, unique destinations, max destination
packets, max destination fan-in.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnsgc.so")

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

NSGC_OK = 0
STATUS = {
    0: "NSGC_OK",
    -1: "NSGC_ERR_INVALID_ARG",
    -2: "NSGC_ERR_BAD_OFFSETS",
    -3: "NSGC_ERR_NO_MEMORY",
    -4: "NSGC_ERR_HIP",
    -5: "NSGC_ERR_INTERNAL",
    -6: "NSGC_ERR_CAPTURING",
    -7: "NSGC_ERR_TOO_LARGE",
}

# Every function declared in include/nsgc.h.
EXPORTS = (
    "nsgc_window_stats",
    "nsgc_window_stats_plain",
    "nsgc_window_stats_timed",
    "nsgc_window_stats_noalloc",
    "nsgc_status_string",
    "nsgc_last_hip_error",
    "nsgc_set_plain_mode",
    "nsgc_get_plain_mode",
    "nsgc_reserve",
    "nsgc_reserve_stream",
    "nsgc_release",
    "nsgc_get_tune",
    "nsgc_set_tune",
    "nsgc_default_tune",
    "nsgc_plan_inspect",
    "nsgc_plan_sizes",
    "nsgc_graph_create",
    "nsgc_graph_launch",
    "nsgc_graph_destroy",
    "nsgc_window_entity_counts",
    "nsgc_window_entities",
    "nsgc_anonymize",
)


class NsgcError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        text = STATUS.get(status, str(status))
        detail = ""
        try:
            detail = _lib().nsgc_status_string(status).decode()
            if status == -4:
                detail += f" (hipError {_lib().nsgc_last_hip_error()})"
        except Exception:  # pragma: no cover
            pass
        super().__init__(f"{what}: {text}: {detail}")


class TuneClass(ctypes.Structure):
    _fields_ = [("link_target", ctypes.c_int32), ("row_target", ctypes.c_int32),
                ("col_target", ctypes.c_int32), ("wave_target", ctypes.c_int32)]


class Tune(ctypes.Structure):
    _fields_ = [
        ("small_max", ctypes.c_int32),
        ("tile_log2", ctypes.c_int32),
        ("link_slots_log2", ctypes.c_int32),
        ("rc_slots_log2", ctypes.c_int32),
        ("blocks_per_cu", ctypes.c_int32),
        ("max_link_buckets_log2", ctypes.c_int32),
        ("max_rc_buckets_log2", ctypes.c_int32),
        ("max_sweeps_log2", ctypes.c_int32),
        ("combine_probes", ctypes.c_int32),
        ("cls", TuneClass * 33),
        ("large_min_log2", ctypes.c_int32),
        ("row_complete", ctypes.c_int32),
    ]

    SCALARS = ("small_max", "tile_log2", "link_slots_log2", "rc_slots_log2",
               "blocks_per_cu", "max_link_buckets_log2", "max_rc_buckets_log2",
               "max_sweeps_log2", "combine_probes", "large_min_log2", "row_complete")

    def to_dict(self) -> dict:
        d = {k: int(getattr(self, k)) for k in self.SCALARS}
        d["cls"] = [[int(c.link_target), int(c.row_target), int(c.col_target), int(c.wave_target)]
                    for c in self.cls]
        return d

    @classmethod
    def from_dict(cls, d: dict) -> "Tune":
        t = cls()
        _check(_lib().nsgc_default_tune(ctypes.byref(t)), "nsgc_default_tune")
        for k in cls.SCALARS:
            if k in d:
                setattr(t, k, int(d[k]))
        for i, row in enumerate(d.get("cls", [])):
            # [link, row, col] or [link, row, col, wave]; a missing wave target keeps its default
            t.cls[i].link_target, t.cls[i].row_target, t.cls[i].col_target = (int(x) for x in row[:3])
            if len(row) > 3:
                t.cls[i].wave_target = int(row[3])
        return t


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                "python paper_2509_03653_amd/_build.py (there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.nsgc_window_stats.argtypes = [vp, vp, vp, i64, vp, vp]
        lib.nsgc_window_stats.restype = i32
        lib.nsgc_window_stats_plain.argtypes = [vp, vp, vp, i64, vp, vp]
        lib.nsgc_window_stats_plain.restype = i32
        lib.nsgc_window_stats_noalloc.argtypes = [vp, vp, vp, i64, vp, vp]
        lib.nsgc_window_stats_noalloc.restype = i32
        lib.nsgc_window_stats_timed.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        lib.nsgc_window_stats_timed.restype = i32
        lib.nsgc_status_string.argtypes = [i32]
        lib.nsgc_status_string.restype = ctypes.c_char_p
        lib.nsgc_last_hip_error.argtypes = []
        lib.nsgc_last_hip_error.restype = i32
        lib.nsgc_set_plain_mode.argtypes = [i32]
        lib.nsgc_set_plain_mode.restype = i32
        lib.nsgc_get_plain_mode.argtypes = []
        lib.nsgc_get_plain_mode.restype = i32
        lib.nsgc_reserve.argtypes = [i64, i64]
        lib.nsgc_reserve.restype = i32
        lib.nsgc_reserve_stream.argtypes = [i64, i64, vp]
        lib.nsgc_reserve_stream.restype = i32
        lib.nsgc_release.argtypes = []
        lib.nsgc_release.restype = i32
        lib.nsgc_get_tune.argtypes = [ctypes.POINTER(Tune)]
        lib.nsgc_get_tune.restype = i32
        lib.nsgc_set_tune.argtypes = [ctypes.POINTER(Tune)]
        lib.nsgc_set_tune.restype = i32
        lib.nsgc_default_tune.argtypes = [ctypes.POINTER(Tune)]
        lib.nsgc_default_tune.restype = i32
        lib.nsgc_plan_inspect.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
        lib.nsgc_plan_inspect.restype = i32
        lib.nsgc_plan_sizes.argtypes = [vp, i64, vp, vp, vp, vp]
        lib.nsgc_plan_sizes.restype = i32
        lib.nsgc_graph_create.argtypes = [i64, i64, ctypes.POINTER(vp)]
        lib.nsgc_graph_create.restype = i32
        lib.nsgc_graph_launch.argtypes = [vp, vp, vp, vp, i64, vp, vp]
        lib.nsgc_graph_launch.restype = i32
        lib.nsgc_graph_destroy.argtypes = [vp]
        lib.nsgc_graph_destroy.restype = i32
        lib.nsgc_window_entity_counts.argtypes = [vp, vp, vp, i64, vp, vp]
        lib.nsgc_window_entity_counts.restype = i32
        lib.nsgc_window_entities.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.nsgc_window_entities.restype = i32
        lib.nsgc_anonymize.argtypes = [vp, vp, i64, ctypes.c_uint64, vp, vp, vp, vp]
        lib.nsgc_anonymize.restype = i32
        _LIB = lib
    return _LIB


def library():
    """The loaded ``libnsgc.so`` (ctypes handle)."""
    return _lib()


def _check(rc: int, what: str):
    if rc != NSGC_OK:
        raise NsgcError(rc, what)


def _offsets(offsets) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))


def _device_u32(t, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on a GPU")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on a GPU (there is no CPU path)")
    if t.dtype not in (torch.int32, torch.uint32):
        raise TypeError(f"{name} must be int32 or uint32 (32-bit addresses)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _stream_handle(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(int(stream.cuda_stream))


def _run(fn, what, src, dst, offsets, out, stream):
    import torch
    src = _device_u32(src, "src")
    dst = _device_u32(dst, "dst")
    if src.device != dst.device:
        raise ValueError("src and dst must be on the same device")
    off = _offsets(offsets)
    w = len(off) - 1
    if w < 0:
        raise ValueError("offsets needs at least one entry")
    if w > 0 and (off[-1] > src.numel() or off[-1] > dst.numel()):
        raise ValueError("offsets run past the packet arrays")
    if out is None:
        out = torch.empty((w, 9), dtype=torch.int64, device=src.device)
    elif out.shape != (w, 9) or out.dtype != torch.int64 or not out.is_contiguous() or out.device != src.device:
        raise ValueError("out must be a contiguous (W, 9) int64 tensor on the packets' device")
    with torch.cuda.device(src.device):
        rc = fn(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                ctypes.c_void_p(off.ctypes.data), w, ctypes.c_void_p(out.data_ptr()),
                _stream_handle(stream, src.device))
    _check(rc, what)
    return out


INVALID_BIT = 1 << 63


def check_valid(stats) -> None:
    """Raise if any window of a finished (W, 9) result carries the library's
    invalid marker (bit 63 of valid_packets).  Synchronises with the tensor."""
    import torch
    col = stats[:, 0] if isinstance(stats, torch.Tensor) else np.asarray(stats)[:, 0]
    bad = (col < 0) if isinstance(stats, torch.Tensor) else (np.asarray(col).astype(np.uint64) >> np.uint64(63)) != 0
    if bool(bad.any()):
        raise NsgcError(-5, "window statistics marked invalid by the library")


def window_stats(src, dst, offsets, out=None, stream=None):
    """Batched form (``nsgc_window_stats``): one (W, 9) int64 tensor, enqueued
    on ``stream`` (default: the current stream)."""
    return _run(_lib().nsgc_window_stats, "nsgc_window_stats", src, dst, offsets, out, stream)


def window_stats_plain(src, dst, offsets, out=None, stream=None):
    """Plain form (``nsgc_window_stats_plain``): one launch sequence per window."""
    return _run(_lib().nsgc_window_stats_plain, "nsgc_window_stats_plain", src, dst, offsets,
                out, stream)


def window_stats_noalloc(src, dst, offsets, out=None, stream=None):
    """Fixed-scratch form (``nsgc_window_stats_noalloc``): the library
    allocates nothing; pass ``out`` to keep the call allocation-free on the
    Python side too.  Batches beyond the fixed scratch raise
    NSGC_ERR_TOO_LARGE."""
    return _run(_lib().nsgc_window_stats_noalloc, "nsgc_window_stats_noalloc", src, dst, offsets,
                out, stream)


# Fixed scratch of nsgc_window_stats_noalloc (include/nsgc.h).
NOALLOC_SCRATCH_BYTES = 128 << 20
NOALLOC_PLAN_BYTES = 2 << 20


PHASES = ("small", "partition", "links", "rowcol", "large")


def window_stats_timed(src, dst, offsets, out=None, stream=None):
    """Measurement form (``nsgc_window_stats_timed``): returns ``(out, phase_ms)``
    with the HIP-event duration of each phase (PHASES)."""
    ms = (ctypes.c_float * len(PHASES))()
    fn = lambda *a: _lib().nsgc_window_stats_timed(*a, ms)  # noqa: E731
    out = _run(fn, "nsgc_window_stats_timed", src, dst, offsets, out, stream)
    return out, dict(zip(PHASES, (float(x) for x in ms)))


def reserve(max_packets: int, max_windows: int, stream=None):
    """Pre-size the workspace of the null stream (``nsgc_reserve``), or of
    ``stream`` when given (``nsgc_reserve_stream``)."""
    if stream is None:
        _check(_lib().nsgc_reserve(int(max_packets), int(max_windows)), "nsgc_reserve")
        return
    _check(_lib().nsgc_reserve_stream(int(max_packets), int(max_windows),
                                      ctypes.c_void_p(int(stream.cuda_stream))),
           "nsgc_reserve_stream")


def set_plain_mode(on: bool):
    """Route ``window_stats`` through the plain one-window-per-launch form."""
    _check(_lib().nsgc_set_plain_mode(1 if on else 0), "nsgc_set_plain_mode")


def plain_mode() -> bool:
    return bool(_lib().nsgc_get_plain_mode())


def release():
    _check(_lib().nsgc_release(), "nsgc_release")


def get_tune() -> Tune:
    t = Tune()
    _check(_lib().nsgc_get_tune(ctypes.byref(t)), "nsgc_get_tune")
    return t


def default_tune() -> Tune:
    t = Tune()
    _check(_lib().nsgc_default_tune(ctypes.byref(t)), "nsgc_default_tune")
    return t


def set_tune(t: Tune):
    _check(_lib().nsgc_set_tune(ctypes.byref(t)), "nsgc_set_tune")


def plan_inspect(offsets) -> dict:
    """Host-only view of the planner's decisions for a batch (no GPU needed)."""
    off = _offsets(offsets)
    w = len(off) - 1
    n = max(w, 1)
    tier = np.zeros(n, np.int32)
    lb = np.zeros(n, np.int32)
    lr = np.zeros(n, np.int32)
    lc = np.zeros(n, np.int32)
    tiles = np.zeros(n, np.int64)
    wsb = np.zeros(1, np.int64)
    rc = _lib().nsgc_plan_inspect(
        ctypes.c_void_p(off.ctypes.data), w, ctypes.c_void_p(tier.ctypes.data),
        ctypes.c_void_p(lb.ctypes.data), ctypes.c_void_p(lr.ctypes.data),
        ctypes.c_void_p(lc.ctypes.data), ctypes.c_void_p(tiles.ctypes.data),
        ctypes.c_void_p(wsb.ctypes.data))
    _check(rc, "nsgc_plan_inspect")
    return {"tier": tier[:w], "log2_link_buckets": lb[:w], "log2_row_buckets": lr[:w],
            "log2_col_buckets": lc[:w], "tiles": tiles[:w], "workspace_bytes": int(wsb[0])}


def plan_sizes(offsets) -> dict:
    """Host-only: the batch's plan and workspace bytes and the bounds used to
    pre-size them for batches of as many packets and windows (no GPU needed)."""
    off = _offsets(offsets)
    v = np.zeros(4, np.int64)
    rc = _lib().nsgc_plan_sizes(ctypes.c_void_p(off.ctypes.data), len(off) - 1,
                                *(ctypes.c_void_p(v.ctypes.data + 8 * k) for k in range(4)))
    _check(rc, "nsgc_plan_sizes")
    return {"plan_bytes": int(v[0]), "workspace_bytes": int(v[1]), "plan_bound": int(v[2]),
            "workspace_bound": int(v[3])}


ENTITY_COUNT_NAMES = ("links", "sources", "destinations", "unique_ips")


def window_entity_counts(src, dst, offsets, out=None, stream=None):
    """Per-window list lengths of the entity outputs and the number of
    globally unique IP addresses (``nsgc_window_entity_counts``): a (W, 4)
    int64 tensor of links, sources, destinations and unique IPs."""
    import torch
    src = _device_u32(src, "src")
    dst = _device_u32(dst, "dst")
    off = _offsets(offsets)
    w = len(off) - 1
    if w > 0 and (off[-1] > src.numel() or off[-1] > dst.numel()):
        raise ValueError("offsets run past the packet arrays")
    if out is None:
        out = torch.empty((max(w, 0), 4), dtype=torch.int64, device=src.device)
    elif out.shape != (w, 4) or out.dtype != torch.int64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous (W, 4) int64 tensor")
    with torch.cuda.device(src.device):
        rc = _lib().nsgc_window_entity_counts(
            ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
            ctypes.c_void_p(off.ctypes.data), w, ctypes.c_void_p(out.data_ptr()),
            _stream_handle(stream, src.device))
    _check(rc, "nsgc_window_entity_counts")
    return out


def window_entities(src, dst, offsets, stream=None):
    """The entity lists of every window (``nsgc_window_entities``), sized by
    a first ``nsgc_window_entity_counts`` call (which synchronises).  Returns a
    dict: ``links`` (L, 3) rows (src, dst, packets), ``sources`` (S, 3) rows
    (s, r(s), f(s)), ``destinations`` (D, 3) rows (d, c(d), g(d)), the
    per-window row offsets of each list (``*_offsets``, numpy int64, W + 1),
    and ``counts`` (W, 4).  Addresses are int64 values of the uint32 addresses;
    rows within a window come in no particular order."""
    import torch
    src = _device_u32(src, "src")
    dst = _device_u32(dst, "dst")
    off = _offsets(offsets)
    w = len(off) - 1
    counts = window_entity_counts(src, dst, off, stream=stream)
    if stream is None:
        torch.cuda.current_stream(src.device).synchronize()
    else:
        stream.synchronize()
    c = counts.cpu().numpy()
    offs = [np.concatenate([[0], np.cumsum(c[:, k])]).astype(np.int64) for k in range(3)]
    lists = [torch.empty((max(int(o[-1]), 0), 3), dtype=torch.int64, device=src.device)
             for o in offs]
    counts2 = torch.empty_like(counts)
    with torch.cuda.device(src.device):
        rc = _lib().nsgc_window_entities(
            ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
            ctypes.c_void_p(off.ctypes.data), w,
            ctypes.c_void_p(offs[0].ctypes.data), ctypes.c_void_p(lists[0].data_ptr()),
            ctypes.c_void_p(offs[1].ctypes.data), ctypes.c_void_p(lists[1].data_ptr()),
            ctypes.c_void_p(offs[2].ctypes.data), ctypes.c_void_p(lists[2].data_ptr()),
            ctypes.c_void_p(counts2.data_ptr()), _stream_handle(stream, src.device))
    _check(rc, "nsgc_window_entities")
    return {"links": lists[0], "sources": lists[1], "destinations": lists[2],
            "link_offsets": offs[0], "source_offsets": offs[1], "destination_offsets": offs[2],
            "counts": counts2}


def anonymize(src, dst, seed: int, out_src=None, out_dst=None, stream=None):
    """Anonymized address columns (``nsgc_anonymize``): every address becomes
    pi(its rank among the unique addresses of both columns in ascending
    order), pi the seeded permutation of [0, N) described in include/nsgc.h.
    Returns ``(anon_src, anon_dst, num_addresses)`` with the counts in a
    one-element int64 tensor (all on the packets' device)."""
    import torch
    src = _device_u32(src, "src")
    dst = _device_u32(dst, "dst")
    if src.numel() != dst.numel():
        raise ValueError("src and dst differ in length")
    out_src = torch.empty_like(src) if out_src is None else _device_u32(out_src, "out_src")
    out_dst = torch.empty_like(dst) if out_dst is None else _device_u32(out_dst, "out_dst")
    if out_src.numel() != src.numel() or out_dst.numel() != dst.numel():
        raise ValueError("outputs must match the inputs' length")
    num = torch.empty(1, dtype=torch.int64, device=src.device)
    with torch.cuda.device(src.device):
        rc = _lib().nsgc_anonymize(
            ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), src.numel(),
            ctypes.c_uint64(int(seed) & (2 ** 64 - 1)), ctypes.c_void_p(out_src.data_ptr()),
            ctypes.c_void_p(out_dst.data_ptr()), ctypes.c_void_p(num.data_ptr()),
            _stream_handle(stream, src.device))
    _check(rc, "nsgc_anonymize")
    return out_src, out_dst, num


class Graph:
    """Reusable captured graph of the batched form (``nsgc_graph_*``)."""

    def __init__(self, max_packets: int, max_windows: int):
        h = ctypes.c_void_p()
        _check(_lib().nsgc_graph_create(int(max_packets), int(max_windows), ctypes.byref(h)),
               "nsgc_graph_create")
        self._h = h

    def launch(self, src, dst, offsets, out=None, stream=None):
        if self._h is None:
            raise RuntimeError("graph destroyed")
        fn = lambda *a: _lib().nsgc_graph_launch(self._h, *a)  # noqa: E731
        return _run(fn, "nsgc_graph_launch", src, dst, offsets, out, stream)

    def close(self):
        if self._h is not None:
            _check(_lib().nsgc_graph_destroy(self._h), "nsgc_graph_destroy")
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass
