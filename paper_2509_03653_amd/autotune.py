"""Autotuner for the batched form.

Every tuning of the library gives identical statistics; only the speed
changes with the batch's size mix and the device.  This module searches the
planner's knobs (LDS-tier cut-over, partition tile, LDS table sizes, resident
workgroups per CU, bucket sizes) for the fastest setting on a given batch,
checks that each tried setting reproduces the baseline statistics bit for
bit, and caches the winner on disk keyed by device and batch shape.

The search is coordinate descent: knobs are visited in a fixed order, every
candidate value of the current knob is timed with the others held, and a
value is kept only if it beats the incumbent by a margin.  `search` is a pure
function of a `measure` callback so that the search loop is testable without a
GPU; `tune_for` supplies the measured callback (captured graph launches timed
with HIP events on the launch stream).
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time
from dataclasses import dataclass, field

import numpy as np

import paper_2509_03653_amd as nsgc

# Knobs in visiting order with their candidate values.  The *_scale knobs
# multiply the per-class bucket targets of every size class present in the
# batch (the other classes keep their defaults): link_scale the link target,
# rc_scale the row and column targets, and row_scale the row target once more
# (sources often repeat more than destinations, so their buckets can be
# larger: on 64 windows of 2^17 Zipf packets, rows of 8192 packets against
# columns of 4096 make phase C 6 us faster, where larger columns overflow).
SPACE = (
    ("blocks_per_cu", (1, 2, 3, 4)),
    ("link_slots_log2", (11, 12)),
    ("rc_slots_log2", (11, 12, 13)),
    ("tile_log2", (12, 13, 14)),
    ("small_max", (256, 512, 1024, 2048)),
    ("link_scale", (0.5, 1.0, 2.0)),
    ("max_link_buckets_log2", (10, 11, 12)),
    ("rc_scale", (0.5, 1.0, 2.0)),
    ("row_scale", (0.5, 1.0, 2.0)),
    ("wave_target", (0, 128, 256, 512)),
    ("combine_probes", (0, 64)),
)

CACHE_VERSION = 4


def size_classes(offsets) -> np.ndarray:
    """Packets per size class k (windows with 2^k <= n < 2^(k+1); class 0 also
    holds empty windows), the planner's own classing."""
    off = np.asarray(offsets, dtype=np.int64)
    n = np.diff(off)
    cls = np.zeros(n.shape, np.int64)
    pos = n > 0
    cls[pos] = np.floor(np.log2(n[pos])).astype(np.int64)
    return np.bincount(cls, weights=n.astype(np.float64), minlength=33)[:33]


def signature(offsets) -> str:
    """Coarse batch shape: total packets and window count (log2, rounded) and
    the packet share of every size class (to 10%).  Batches with the same
    signature share a cached tuning."""
    off = np.asarray(offsets, dtype=np.int64)
    w = len(off) - 1
    total = int(off[-1] - off[0]) if w > 0 else 0
    pc = size_classes(off)
    share = pc / max(total, 1)
    mix = ",".join(f"{k}:{round(s * 10)}" for k, s in enumerate(share) if round(s * 10) > 0)
    return f"p{round(math.log2(total + 1))}-w{round(math.log2(w + 1))}-[{mix}]"


def device_key(device=None) -> str:
    """Architecture, compute-unit count, HIP runtime and library build."""
    import torch
    dev = torch.cuda.current_device() if device is None else device
    prop = torch.cuda.get_device_properties(dev)
    arch = getattr(prop, "gcnArchName", prop.name)
    with open(nsgc.LIB_PATH, "rb") as f:
        lib = hashlib.sha1(f.read()).hexdigest()[:12]
    return f"{arch}-cu{prop.multi_processor_count}-hip{torch.version.hip}-lib{lib}"


def default_cache_path() -> str:
    return os.environ.get("NSGC_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "nsgc", "tune.json"))


# ---- tunings as plain dicts -------------------------------------------------

def apply_point(base: dict, point: dict, classes) -> dict:
    """The full tuning dict for a search point: scalar knobs replace the base
    values, *_scale knobs scale the targets of the given size classes."""
    d = json.loads(json.dumps(base))
    for k, v in point.items():
        if k in ("link_scale", "rc_scale", "row_scale"):
            continue
        if k == "wave_target":
            for c in classes:
                d["cls"][c][3] = int(v)
        else:
            d[k] = v
    # the scales in a fixed order (row_scale applies on top of rc_scale)
    for c in classes:
        d["cls"][c][0] = max(64, int(d["cls"][c][0] * point.get("link_scale", 1.0)))
        rc = point.get("rc_scale", 1.0)
        d["cls"][c][1] = max(64, int(d["cls"][c][1] * rc * point.get("row_scale", 1.0)))
        d["cls"][c][2] = max(64, int(d["cls"][c][2] * rc))
    return d


def start_point(base: dict) -> dict:
    p = {k: base[k] for k, _ in SPACE if k in base}
    p["link_scale"] = 1.0
    p["rc_scale"] = 1.0
    p["row_scale"] = 1.0
    waves = {row[3] for row in base["cls"] if len(row) > 3}
    if len(waves) == 1:
        p["wave_target"] = waves.pop()
    return p


@dataclass
class SearchResult:
    point: dict
    ms: float
    start_ms: float
    trials: list = field(default_factory=list)   # (point, ms) in the order tried


def search(measure, start: dict, space=SPACE, margin=0.02, max_trials=64,
           budget_s=None, clock=time.monotonic) -> SearchResult:
    """Coordinate descent over `space` from `start`.

    `measure(point) -> ms` returns the time of one batched step for the point
    (or raises).  A candidate replaces the incumbent only when it is faster
    by more than `margin` (relative).  Stops after `max_trials` measurements
    or `budget_s` seconds.
    """
    t0 = clock()
    best = dict(start)
    best_ms = float(measure(best))
    res = SearchResult(point=best, ms=best_ms, start_ms=best_ms, trials=[(dict(best), best_ms)])
    for knob, values in space:
        for v in values:
            if len(res.trials) >= max_trials or (budget_s is not None and clock() - t0 > budget_s):
                res.point, res.ms = best, best_ms
                return res
            if best.get(knob) == v:
                continue
            cand = dict(best)
            cand[knob] = v
            ms = float(measure(cand))
            res.trials.append((dict(cand), ms))
            if ms < best_ms * (1.0 - margin):
                best, best_ms = cand, ms
    res.point, res.ms = best, best_ms
    return res


# ---- cache ------------------------------------------------------------------

def cache_load(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    if data.get("version") != CACHE_VERSION:
        return {}
    return data.get("entries", {})


def cache_store(path: str, key: str, entry: dict) -> None:
    entries = cache_load(path)
    entries[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump({"version": CACHE_VERSION, "entries": entries}, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cached(offsets, cache_path=None, device=None):
    """The cached tuning for this device and batch shape, or None."""
    e = cache_load(cache_path or default_cache_path()).get(
        f"{device_key(device)}|{signature(offsets)}")
    return nsgc.Tune.from_dict(e["tune"]) if e else None


# ---- measured search on the GPU ---------------------------------------------

class MismatchError(AssertionError):
    """A tuning produced statistics different from the baseline's."""


def _time_graph(tune_dict, src, dst, off, repeats, warmup, want, stream):
    import torch
    nsgc.set_tune(nsgc.Tune.from_dict(tune_dict))
    w = len(off) - 1
    g = nsgc.Graph(max(int(off[-1] - off[0]), 1), max(w, 1))
    try:
        out = torch.empty((w, 9), dtype=torch.int64, device=src.device)
        for _ in range(warmup):
            g.launch(src, dst, off, out=out, stream=stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(repeats + 1)]
        ev[0].record(stream)
        for i in range(repeats):
            g.launch(src, dst, off, out=out, stream=stream)
            ev[i + 1].record(stream)
        stream.synchronize()
        ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(repeats))
        if want is not None and not torch.equal(out, want):
            raise MismatchError(f"tuning {tune_dict} changed the statistics")
        return ms[len(ms) // 2], out
    finally:
        g.close()


def tune_for(src, dst, offsets, *, cache_path=None, force=False, apply=True, repeats=5,
             warmup=2, max_trials=40, budget_s=60.0, space=SPACE, margin=0.02):
    """Find (or load) the fastest tuning for this batch shape on this device.

    `src`/`dst` are device tensors holding a representative batch.  Returns
    a dict with the tuning, its time, the default's time and whether it came
    from the cache; installs the tuning when `apply`.
    """
    import torch
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    path = cache_path or default_cache_path()
    key = f"{device_key(src.device.index)}|{signature(off)}"
    if not force:
        e = cache_load(path).get(key)
        if e is not None:
            if apply:
                nsgc.set_tune(nsgc.Tune.from_dict(e["tune"]))
            return dict(e, cached=True, key=key)

    before = nsgc.get_tune()
    base = nsgc.default_tune().to_dict()
    pc = size_classes(off)
    classes = [k for k in range(33) if pc[k] > 0]
    stream = torch.cuda.current_stream(src.device)
    try:
        _, want = _time_graph(base, src, dst, off, 1, 1, None, stream)

        def measure(point):
            ms, _ = _time_graph(apply_point(base, point, classes), src, dst, off, repeats,
                                warmup, want, stream)
            return ms

        res = search(measure, start_point(base), space=space, margin=margin,
                     max_trials=max_trials, budget_s=budget_s)
    except BaseException:
        nsgc.set_tune(before)
        raise
    best = apply_point(base, res.point, classes)
    entry = {"tune": best, "ms": res.ms, "default_ms": res.start_ms, "point": res.point,
             "trials": len(res.trials), "signature": signature(off)}
    cache_store(path, key, entry)
    nsgc.set_tune(nsgc.Tune.from_dict(best) if apply else before)
    return dict(entry, cached=False, key=key)
