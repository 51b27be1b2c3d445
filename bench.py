#!/usr/bin/env python3
"""Throughput of the per-window statistics hot path on one MI355X.

Workload: 64 windows x 2^17 packets, src Zipf(1.2) over 2^20 addresses, dst
Zipf(1.0) over 2^24 addresses (seeded synthetic stand-in for one archive of
the paper's capture: 64 matrices of 2^17 packets, Section IV "GraphBLAS
format").  A step is one pass of the whole hot path (plan, partition, link
aggregation, row/column aggregation, reductions) over the batch; inputs are
resident in HBM before the timed region, and the step rotates over 8 copies
of the input (537 MB > the 256 MB Infinity Cache), so the packets come from
HBM, not the cache.

Prints ONE JSON line.  Also reports the plain one-window-per-launch form, the
direct (uncaptured) batched form, per-kernel HIP-event times with the roofline
of the dominant kernel, the CPU oracle as a baseline on a bounded sample, and
a serving leg: continuous batching of Poisson-arriving windows (log-uniform
2^12..2^22 packets) with p50/p99 latency at three offered rates.

Extra modes:
  --profile-steps N   only run N batched graph steps plus one calibration copy
                      of known size (for rocprofv3 counter runs)
  --summarize-pmc FETCH_DIR WRITE_DIR
                      turn two rocprofv3 --pmc runs into profiles/ summaries
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0                     # MI355X HBM3E, 8 TB/s
COPIES = 8
CALIB_BYTES = 1 << 30                     # calibration copy: 1 GiB read + 1 GiB written
# measured HBM traffic per workload (written by --summarize-pmc), keyed by kernel sources
TRAFFIC_NAMES = {"zipf_batch": "zipf_64x2^17", "uniform_single": "uniform_1x2^17",
                 "skewed_large": "skewed_128x2^23", "uneven_batch": "uneven_4096"}


def traffic_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{TRAFFIC_NAMES[workload]}.json")


def measured_traffic(workload: str, phase: str):
    """HBM bytes per launch of `phase` from the stored counters, or None when
    none were taken or the kernel sources have changed since."""
    f = traffic_file(workload)
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        tr = json.load(fh)
    if tr.get("kernel_source") != kernel_source_hash() or phase not in tr.get("phases", {}):
        return None
    return tr["phases"][phase]["hbm_bytes"]
# the launches each timed phase covers (the link phase is one of two kernels,
# the row/column phase includes the ordering and the per-window combine)
PHASE_KERNELS = {"small": ["k_small"], "partition": ["k_partition"],
                 "links": ["k_links_wave", "k_links"],
                 "rowcol": ["k_order", "k_rowcol", "k_finish"]}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2509_03653_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(num_packets: int, num_windows: int) -> int:
    # 8 B per packet read (src + dst) + 8 B of offsets and 72 B of statistics per window
    return 8 * num_packets + 80 * num_windows


WORKLOAD_TEXT = {
    "zipf_batch": "64 windows x 2^17 packets, src Zipf(1.2) over 2^20 addresses, "
                  "dst Zipf(1.0) over 2^24 addresses",
    "uniform_single": "1 window x 2^17 packets, src and dst uniform over 4096 addresses",
    "skewed_large": "128 windows x 2^23 packets, 10% from one super-source, 1% to one "
                    "super-destination, rest Zipf(1.3) over 2^26 addresses",
    "uneven_batch": "4096 windows, sizes log-uniform in [2^10, 2^23], Zipf(1.1) over 2^22 "
                    "addresses",
}


def tune_with(nsgc, spec: str):
    """The default tuning with `key=value` overrides (comma-separated)."""
    t = nsgc.default_tune()
    per_class = ("link_target", "row_target", "col_target", "wave_target")
    for kv in filter(None, spec.split(",")):
        k, v = kv.split("=")
        if k in per_class:
            for c in t.cls:
                setattr(c, k, int(v))
        elif k in nsgc.Tune.SCALARS:
            setattr(t, k, int(v))
        else:
            raise SystemExit(f"unknown tuning knob {k!r}")
    return t


def synth_workload(name, seed):
    import synth
    return synth.WORKLOADS[name](seed=seed)


def stream_copy_gbs(torch, stream, nbytes=CALIB_BYTES, reps=5):
    """Device-to-device copy bandwidth (bytes read + written per second) of a
    1 GiB buffer: what a plain streaming kernel reaches on this device."""
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    ms = time_loop(lambda i: b.copy_(a), reps, 2, stream)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def make_inputs(args):
    import synth
    wl = synth.WORKLOADS[args.workload](seed=args.seed)
    src, dst = wl.generate()
    return wl, src, dst


def sample_windows(num_windows: int):
    return sorted({0, num_windows // 3, (2 * num_windows) // 3, num_windows - 1})


def oracle_on(src, dst, offsets, windows, threads):
    """The oracle on selected windows (gathered into one batch)."""
    import oracle
    parts = [(int(offsets[w]), int(offsets[w + 1])) for w in windows]
    s = np.concatenate([src[a:b] for a, b in parts])
    d = np.concatenate([dst[a:b] for a, b in parts])
    off = np.concatenate([[0], np.cumsum([b - a for a, b in parts])]).astype(np.int64)
    return oracle.window_stats(s, d, off, threads=threads)


def to_device_copies(src, dst, copies):
    import torch
    s = torch.from_numpy(src.view(np.int32)).cuda()
    d = torch.from_numpy(dst.view(np.int32)).cuda()
    ss, dd = [s], [d]
    for _ in range(copies - 1):
        ss.append(s.clone())
        dd.append(d.clone())
    torch.cuda.synchronize()
    return ss, dd


def time_loop(fn, steps, warmup, stream):
    import torch
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for i in range(steps):
        fn(i)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    return "unknown"


def oracle_single_thread(src, dst, offsets, budget_s: float):
    """The oracle on one core over the whole batch (repeated within the
    budget): packets/s."""
    import oracle
    n_all = int(offsets[-1] - offsets[0])
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.window_stats(src, dst, offsets, threads=1)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 20:
            break
    return n_all * reps / el


def latency_leg(nsgc, torch, seed, calls=200):
    """One window of 2^17 packets uniform over 4096 addresses: microseconds
    per call of the graph form and of the direct batched form, each a loop
    of back-to-back calls on one stream (launch-bound)."""
    import synth
    wl = synth.uniform_single(seed=seed)
    src, dst = wl.generate()
    off = wl.offsets
    s = torch.from_numpy(src.view(np.int32)).cuda()
    d = torch.from_numpy(dst.view(np.int32)).cuda()
    out = torch.empty((1, 9), dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    g = nsgc.Graph(wl.num_packets, 1)
    try:
        g.launch(s, d, off, out=out, stream=stream)
        torch.cuda.synchronize()
        import oracle
        if not np.array_equal(out.cpu().numpy().view(np.uint64), oracle.window_stats(src, dst, off)):
            raise SystemExit("parity check failed on the single uniform window")
        ms_g = time_loop(lambda i: g.launch(s, d, off, out=out, stream=stream), calls, 20, stream)
        ms_d = time_loop(lambda i: nsgc.window_stats(s, d, off, out=out, stream=stream), calls, 20,
                         stream)
    finally:
        g.close()
    st1 = oracle_single_thread(src, dst, off, 2.0)
    return {"workload": WORKLOAD_TEXT["uniform_single"], "packets": wl.num_packets,
            "graph_us_per_call": ms_g * 1e3, "direct_us_per_call": ms_d * 1e3,
            "graph_packets_per_s": wl.num_packets / (ms_g * 1e-3),
            "direct_packets_per_s": wl.num_packets / (ms_d * 1e-3),
            "oracle_single_thread_packets_per_s": st1}


def large_leg(nsgc, torch, seed, steps=5):
    """128 windows of 2^23 skewed packets (2^30 in total): batched graph and
    plain per-window forms, per-phase times and the dominant kernel's
    roofline; parity-gated on four windows first."""
    import synth
    wl = synth.skewed_large(seed=seed)
    src, dst = wl.generate()
    off = wl.offsets
    P, W = wl.num_packets, wl.num_windows
    s = torch.from_numpy(src.view(np.int32)).cuda()
    d = torch.from_numpy(dst.view(np.int32)).cuda()
    out = torch.empty((W, 9), dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    g = nsgc.Graph(P, W)
    try:
        g.launch(s, d, off, out=out, stream=stream)
        torch.cuda.synchronize()
        sample = sample_windows(W)
        want = oracle_on(src, dst, off, sample, threads=len(sample))
        if not np.array_equal(out.cpu().numpy().view(np.uint64)[sample], want):
            raise SystemExit("parity check failed on the skewed 2^30-packet batch")
        ms_g = time_loop(lambda i: g.launch(s, d, off, out=out, stream=stream), steps, 2, stream)
    finally:
        g.close()
    ms_p = time_loop(lambda i: nsgc.window_stats_plain(s, d, off, out=out, stream=stream),
                     max(steps // 2, 2), 1, stream)
    phases = {k: [] for k in nsgc.PHASES}
    for _ in range(steps):
        _, ph = nsgc.window_stats_timed(s, d, off, out=out, stream=stream)
        for k, v in ph.items():
            phases[k].append(v)
    phase_ms = {k: float(np.mean(v)) for k, v in phases.items()}
    dom = max(phase_ms, key=phase_ms.get)
    alg = algorithmic_bytes(P, W)
    ach = alg / (phase_ms[dom] * 1e-3) / 1e9
    del s, d
    torch.cuda.empty_cache()
    nsgc.release()
    return {"workload": WORKLOAD_TEXT["skewed_large"], "windows": W, "packets": P,
            "batched_ms_per_step": ms_g, "batched_packets_per_s": P / (ms_g * 1e-3),
            "plain_ms_per_step": ms_p, "plain_packets_per_s": P / (ms_p * 1e-3),
            "batched_over_plain": ms_p / ms_g, "phase_ms": phase_ms,
            "step_roofline_frac": alg / (ms_g * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "roofline": {"bound": "hbm", "phase": dom, "kernels": PHASE_KERNELS[dom],
                         "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS,
                         "traffic": measured_traffic("skewed_large", dom)}}


def single_large_leg(nsgc, torch, seed, steps=3):
    """One window of 2^30 skewed packets (the whole capture as one graph):
    the large-window tier, direct batched form, per-phase times; checked by
    the statistics' invariants and the src/dst swap relation first (the
    oracle would need minutes for it)."""
    import synth
    wl = synth.skewed_large(seed=seed, num_windows=1, log2_window=30)
    src, dst = wl.generate()
    off = wl.offsets
    n = wl.num_packets
    s = torch.from_numpy(src.view(np.int32)).cuda()
    d = torch.from_numpy(dst.view(np.int32)).cuda()
    del src, dst
    stream = torch.cuda.current_stream()
    fwd = nsgc.window_stats(s, d, off, stream=stream)
    rev = nsgc.window_stats(d, s, off, stream=stream)
    torch.cuda.synchronize()
    a = fwd.cpu().numpy().view(np.uint64)[0]
    b = rev.cpu().numpy().view(np.uint64)[0]
    ok = (int(a[0]) == n and np.array_equal(b, a[[0, 1, 2, 6, 7, 8, 3, 4, 5]])
          and a[1] <= a[0] and a[3] <= a[1] and a[6] <= a[1] and a[4] <= a[0]
          and a[5] <= a[6] and a[8] <= a[3] and a[2] <= min(a[4], a[7]))
    if not ok:
        raise SystemExit("invariant check failed on the single 2^30-packet window")
    out = torch.empty((1, 9), dtype=torch.int64, device="cuda")
    ms = time_loop(lambda i: nsgc.window_stats(s, d, off, out=out, stream=stream), steps, 1,
                   stream)
    _, ph = nsgc.window_stats_timed(s, d, off, out=out, stream=stream)
    del s, d
    torch.cuda.empty_cache()
    nsgc.release()
    return {"workload": "1 window x 2^30 packets, 10% from one super-source, 1% to one "
                        "super-destination, rest Zipf(1.3) over 2^26 addresses",
            "packets": n, "tier": "large (radix sort)", "ms_per_call": ms,
            "packets_per_s": n / (ms * 1e-3), "phase_ms": ph,
            "algorithmic_frac": 8 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "stats": [int(x) for x in a]}


def cpu_baseline(src, dst, offsets, budget_s: float):
    """The oracle on the host cores: the whole batch, repeated while within
    budget; for batches too large for the budget, consecutive groups of
    windows (one window per thread) until the budget is spent."""
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cores = os.cpu_count() or 1
    W = len(offsets) - 1
    n_all = int(offsets[-1] - offsets[0])
    if n_all <= 64 << 20:
        threads = max(1, min(cores, W))
        reps, t0 = 0, time.perf_counter()
        while True:
            oracle.window_stats(src, dst, offsets, threads=threads)
            reps += 1
            el = time.perf_counter() - t0
            if el >= budget_s or reps >= 50:
                break
        return {"value": n_all * reps / el, "unit": "packets/s", "cores": threads,
                "kind": "oracle",
                "sample": f"the full batch ({W} windows, {n_all} packets) run {reps}x "
                          f"({el:.1f} s wall) with one window per thread"}
    threads = cores
    done_w, done_p, t0 = 0, 0, time.perf_counter()
    while done_w < W:
        group = range(done_w, min(W, done_w + 8 * threads))   # dynamic scheduling balances
        a, b = int(offsets[group[0]]), int(offsets[group[-1] + 1])
        oracle.window_stats(src[a:b], dst[a:b], offsets[group[0]:group[-1] + 2] - a,
                            threads=threads)
        done_w, done_p = group[-1] + 1, done_p + (b - a)
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": done_p / el, "unit": "packets/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {done_w} of {W} windows ({done_p} packets, {el:.1f} s wall) "
                      f"with one window per thread"}


def cpu_baseline_full(src, dst, offsets, budget_s: float):
    r = cpu_baseline(src, dst, offsets, budget_s)
    r["cpu_model"] = cpu_model()
    r["single_thread_value"] = oracle_single_thread(src, dst, offsets, min(budget_s, 6.0))
    return r


def counter_rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    out = []
    for f in files:
        with open(f) as fh:
            out.extend(csv.DictReader(fh))
    return out


def summarize_counters(d):
    """Mean per dispatch of every counter in a rocprofv3 --pmc run, per library
    kernel, as one JSON object {kernel: {counter: value}}."""
    import re
    acc = {}
    for r in counter_rows(d):
        m = re.search(r"nsgc::(k_\w+)", r["Kernel_Name"])
        if not m:
            continue
        disp = r.get("Dispatch_Id", r.get("Correlation_Id"))
        k = acc.setdefault(m.group(1), {}).setdefault(r["Counter_Name"], {})
        k[disp] = k.get(disp, 0.0) + float(r["Counter_Value"])
    res = {kern: {c: float(np.mean(list(v.values()))) for c, v in sorted(cs.items())}
           for kern, cs in sorted(acc.items())}
    print(json.dumps(res, indent=1))


def summarize_pmc(fetch_dir, write_dir, workload="zipf_batch"):
    """Scale FETCH_SIZE / WRITE_SIZE per dispatch by the calibration copy and
    sum them per timed phase (the kernels of PHASE_KERNELS)."""
    import re

    def per_kernel(d, counter):
        acc = {}
        for r in counter_rows(d):
            if r.get("Counter_Name") != counter:
                continue
            name = r["Kernel_Name"]
            m = re.search(r"nsgc::(k_\w+)", name)
            if m:
                key = m.group(1)
            elif "copy" in name.lower() or "elementwise" in name.lower():
                key = "copies"
            else:
                continue
            acc.setdefault(key, {})
            disp = r.get("Dispatch_Id", r.get("Correlation_Id"))
            acc[key][disp] = acc[key].get(disp, 0.0) + float(r["Counter_Value"])
        res = {k: float(np.mean(list(v.values()))) for k, v in acc.items() if k != "copies"}
        if "copies" in acc:   # the calibration copy is by far the largest copy dispatch
            res["calibration_copy"] = float(max(acc["copies"].values()))
        return res

    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")
    cal_f = fetch.get("calibration_copy")
    cal_w = write.get("calibration_copy")
    f_scale = (CALIB_BYTES / 1024.0) / cal_f if cal_f else None
    w_scale = (CALIB_BYTES / 1024.0) / cal_w if cal_w else None
    result = {"kernel_source": kernel_source_hash(), "calibration_bytes": CALIB_BYTES,
              "fetch_scale": f_scale, "write_scale": w_scale, "kernels": {}, "phases": {}}
    for k in sorted(set(fetch) | set(write)):
        if k == "calibration_copy":
            continue
        fb = fetch.get(k, 0.0) * 1024.0 * (f_scale or 1.0)
        wb = write.get(k, 0.0) * 1024.0 * (w_scale or 1.0)
        result["kernels"][k] = {"fetch_kib_raw": fetch.get(k), "write_kib_raw": write.get(k),
                                "hbm_bytes": fb + wb}
    for ph, ks in PHASE_KERNELS.items():
        got = [result["kernels"][k]["hbm_bytes"] for k in ks if k in result["kernels"]]
        if got:
            result["phases"][ph] = {"hbm_bytes": float(sum(got)),
                                    "kernels": [k for k in ks if k in result["kernels"]]}
    result["workload"] = WORKLOAD_TEXT[workload]
    path = traffic_file(workload)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(result, fh, indent=1)
    print(json.dumps(result))


def serving_leg(args, nsgc, torch):
    """Continuous-batching server over Poisson arrivals (windows log-uniform in
    [2^12, 2^22] packets, Zipf(1.2) over 2^24 addresses): the closed-loop
    saturation rate, then open-loop runs at 0.5, 0.8 and 1.0 of it.  Requests
    are served from a pool of generated windows in pinned host memory;
    latency runs from arrival to statistics on the host."""
    import synth
    from paper_2509_03653_amd import serving as sv

    pool_n = args.serving_pool
    wl = synth.serving_stream(seed=args.seed, num_windows=pool_n)
    src, dst = wl.generate()
    off = wl.offsets
    src_pin = torch.from_numpy(src.view(np.int32)).pin_memory()
    dst_pin = torch.from_numpy(dst.view(np.int32)).pin_memory()
    # reference: the pool windows in one batched call
    ref = nsgc.window_stats(src_pin.cuda(), dst_pin.cuda(), off)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy().view(np.uint64)

    cap = 1 << 27
    ex = sv.GpuExecutor(cap, max_batch_windows=1024, streams=2)
    n_total = args.serving_warmup + args.serving_windows

    def requests():
        out = []
        for i in range(n_total):
            k = i % pool_n
            a, b = int(off[k]), int(off[k + 1])
            r = sv.Request(i, src_pin[a:b], dst_pin[a:b])
            r.pool = k
            out.append(r)
        return out

    def serve(times):
        srv = sv.Server(ex, cap, inflight=2, max_batch_windows=1024)
        res = srv.run(requests(), arrival_times=times, warmup=args.serving_warmup, timeout_s=300)
        for r in res.requests:
            if not np.array_equal(r.stats, ref[r.pool]):
                raise SystemExit(f"served window {r.rid} differs from the same window alone")
        return res.summary()

    serve(None)                                   # warm-up of streams and workspaces
    sat = serve(None)
    lam = sat["windows_per_s"]
    rates = []
    for frac in (0.5, 0.8, 1.0):
        s = serve(sv.poisson_arrivals(n_total, frac * lam, seed=args.seed + int(frac * 10)))
        rates.append({"fraction_of_saturation": frac, "offered_windows_per_s": frac * lam,
                      "windows_per_s": s["windows_per_s"], "packets_per_s": s["packets_per_s"],
                      "p50_ms": s["p50_ms"], "p99_ms": s["p99_ms"],
                      "mean_batch_windows": s["mean_batch_windows"]})
    return {"workload": "Poisson arrivals, windows log-uniform in [2^12, 2^22] packets, "
                        "Zipf(1.2) over 2^24 addresses",
            "pool_windows": pool_n, "windows_per_rate": args.serving_windows,
            "warmup_windows": args.serving_warmup, "arena_packets": cap,
            "saturation": {"windows_per_s": lam, "packets_per_s": sat["packets_per_s"],
                           "p50_ms": sat["p50_ms"], "p99_ms": sat["p99_ms"]},
            "rates": rates, "exact": True}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workload", default="zipf_batch", choices=sorted(WORKLOAD_TEXT),
                    help="batch to time (default: 64 windows x 2^17 Zipf packets)")
    ap.add_argument("--autotune", action="store_true",
                    help="search (or load from the cache) the tuning for this batch first")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle wall time for the CPU baseline (0 disables)")
    ap.add_argument("--serving-windows", type=int, default=2000,
                    help="measured windows per offered rate of the serving leg (0 disables)")
    ap.add_argument("--serving-warmup", type=int, default=200)
    ap.add_argument("--serving-pool", type=int, default=256)
    ap.add_argument("--profile-steps", type=int, default=0)
    ap.add_argument("--no-extra-legs", action="store_true",
                    help="skip the single-window latency and the 2^30-packet legs")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-counters", metavar="PMC_DIR",
                    help="print the per-kernel mean of every counter of a rocprofv3 --pmc run")
    ap.add_argument("--tune", default="",
                    help="tuning overrides, e.g. 'max_link_buckets_log2=11,wave_target=0' "
                         "(per-class targets apply to every size class)")
    args = ap.parse_args()

    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, workload=args.workload)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the statistics of independent windows need no "
              f"communication between GPUs, so whole-job throughput on N GPUs is N times the "
              f"one-GPU figure for equal shares (asked for --gpus {args.gpus}; run with --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2509_03653_amd as nsgc

    torch.cuda.set_device(0)
    if args.tune:
        nsgc.set_tune(tune_with(nsgc, args.tune))
    wl, src, dst = make_inputs(args)
    off = wl.offsets
    P, W = wl.num_packets, wl.num_windows
    copies = COPIES if P * 8 * COPIES <= (4 << 30) else 1   # big batches exceed the caches anyway
    ss, dd = to_device_copies(src, dst, copies)
    stream = torch.cuda.current_stream()
    out = torch.empty((W, 9), dtype=torch.int64, device="cuda")
    tuned = None
    if args.autotune:   # before the timed graph: each trial holds a workspace of its own
        from paper_2509_03653_amd import autotune
        tuned = autotune.tune_for(ss[0], dd[0], off, budget_s=120.0)
        nsgc.release()
    graph = nsgc.Graph(P, W)          # a graph keeps the tuning it was created with

    if args.profile_steps:
        for i in range(args.profile_steps):
            graph.launch(ss[i % copies], dd[i % copies], off, out=out, stream=stream)
            nsgc.window_stats(ss[i % copies], dd[i % copies], off, out=out, stream=stream)
        torch.cuda.synchronize()
        a = torch.empty(CALIB_BYTES // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"profile run done: {args.profile_steps} steps + {CALIB_BYTES} B calibration copy",
              flush=True)
        graph.close()
        return


    # parity gate on sampled windows before timing
    graph.launch(ss[0], dd[0], off, out=out, stream=stream)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint64)
    sample = sample_windows(W)
    want = oracle_on(src, dst, off, sample, threads=len(sample))
    if not np.array_equal(got[sample], want):
        raise SystemExit("parity check failed before timing")

    def step_graph(i):
        graph.launch(ss[i % copies], dd[i % copies], off, out=out, stream=stream)

    def step_direct(i):
        nsgc.window_stats(ss[i % copies], dd[i % copies], off, out=out, stream=stream)

    def step_plain(i):
        nsgc.window_stats_plain(ss[i % copies], dd[i % copies], off, out=out, stream=stream)

    ms_graph = time_loop(step_graph, args.steps, args.warmup, stream)
    ms_direct = time_loop(step_direct, args.steps, args.warmup, stream)
    ms_plain = time_loop(step_plain, max(args.steps // 4, 5), max(args.warmup // 2, 2), stream)
    # warm: the same input copy every step (its keys may stay in the 256 MB cache)
    ms_warm = time_loop(lambda i: graph.launch(ss[0], dd[0], off, out=out, stream=stream),
                        args.steps, args.warmup, stream)
    copy_gbs = stream_copy_gbs(torch, stream)
    seed_ms = {str(args.seed): ms_graph}
    if args.workload == "zipf_batch" and not args.tune and not args.autotune:
        for sd in (args.seed + 1, args.seed + 2):   # two more seeds of the same workload
            wl2 = synth_workload(args.workload, sd)
            s2, d2 = wl2.generate()
            a2 = torch.from_numpy(s2.view(np.int32)).cuda()
            b2 = torch.from_numpy(d2.view(np.int32)).cuda()
            seed_ms[str(sd)] = time_loop(
                lambda i: graph.launch(a2, b2, wl2.offsets, out=out, stream=stream),
                args.steps, args.warmup, stream)
            del a2, b2

    # per-kernel HIP-event times on the launch stream
    phases = {k: [] for k in nsgc.PHASES}
    for i in range(args.steps):
        _, ph = nsgc.window_stats_timed(ss[i % copies], dd[i % copies], off, out=out, stream=stream)
        for k, v in ph.items():
            phases[k].append(v)
    phase_ms = {k: float(np.mean(v)) for k, v in phases.items()}
    dominant = max(phase_ms, key=phase_ms.get)
    alg = algorithmic_bytes(P, W)
    achieved = alg / (phase_ms[dominant] * 1e-3) / 1e9

    traffic = None if args.tune or args.autotune else measured_traffic(args.workload, dominant)

    serving = None
    if args.serving_windows > 0 and args.workload == "zipf_batch":
        serving = serving_leg(args, nsgc, torch)

    cpu = None
    if args.cpu_budget > 0:
        cpu = cpu_baseline_full(src, dst, off, args.cpu_budget)

    extra = {}
    if not args.no_extra_legs and args.workload == "zipf_batch":
        extra["single_window"] = latency_leg(nsgc, torch, args.seed)
        del ss, dd
        torch.cuda.empty_cache()
        nsgc.release()
        extra["skewed_2e30"] = large_leg(nsgc, torch, args.seed)
        extra["single_window_2e30"] = single_large_leg(nsgc, torch, args.seed)

    value = P / (ms_graph * 1e-3)
    line = {
        "metric": "packets/sec exact window stats (batched vs plain), % HBM roofline, p99 latency",
        "value": value,
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_graph,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": f"synthetic (seeded traffic; inputs resident in HBM, {copies} rotating "
                f"cop{'ies' if copies > 1 else 'y'})",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "windows": W, "packets": P, "seed": args.seed, "form": "batched, graph",
                   "tuning": "autotuned" if args.autotune else (args.tune or "default")},
        "batched_direct_packets_per_s": P / (ms_direct * 1e-3),
        "plain_packets_per_s": P / (ms_plain * 1e-3),
        "plain_ms_per_step": ms_plain,
        "batched_over_plain": ms_plain / ms_graph,
        "step_algorithmic_GBs": alg / (ms_graph * 1e-3) / 1e9,
        "step_roofline_frac": alg / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "warm_ms_per_step": ms_warm,
        "stream_copy_GBs": copy_gbs,
        "step_frac_of_stream_copy": alg / (ms_graph * 1e-3) / 1e9 / copy_gbs,
        "seed_ms_per_step": seed_ms,
        "seed_median_packets_per_s": P / (float(np.median(list(seed_ms.values()))) * 1e-3),
        "phase_ms": phase_ms,
        "roofline": {"bound": "hbm", "phase": dominant, "kernels": PHASE_KERNELS[dominant],
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "cpu_baseline": cpu,
        "serving": serving,
    }
    line.update(extra)
    if tuned is not None:
        line["autotune"] = {"tune": tuned["tune"], "default_ms": tuned.get("default_ms"),
                            "tuned_ms": tuned.get("ms"), "cached": tuned.get("cached")}
    graph.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
