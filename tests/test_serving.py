"""Serving loop: the ring arena and the continuous-batching scheduler on the
CPU (with an executor that computes each batch from the arena contents at
launch time), and the device executor on the GPU."""
import numpy as np
import pytest

import oracle
import synth
from paper_2509_03653_amd import serving as sv


# ---- ring arena ---------------------------------------------------------------

def test_arena_fifo_alloc_wrap_and_full():
    a = sv.RingArena(10)
    assert a.alloc(4) == 0 and a.alloc(4) == 4
    assert a.alloc(3) is None                 # 2 left at the end, 0 at the front
    a.mark_done(0, 4)
    a.release()
    assert a.alloc(3) == 0                    # wraps; [8, 10) is skipped
    assert a.in_use() == 4 + 2 + 3
    assert a.alloc(2) is None                 # [3, 4) free only: too small
    assert a.alloc(1) == 3
    assert a.alloc(1) is None                 # full
    a.mark_done(3, 1)                         # done out of order: not released yet
    assert a.release() == 0
    a.mark_done(4, 4)
    assert a.release() == 1                   # frees [4, 8) and the skipped tail
    a.mark_done(0, 3)
    assert a.release() == 2
    assert a.in_use() == 0 and a.alloc(10) == 0
    with pytest.raises(ValueError):
        a.alloc(11)
    with pytest.raises(ValueError):
        a.alloc(0)


def test_arena_random_workload_never_overlaps():
    rng = np.random.default_rng(5)
    cap = 1000
    a = sv.RingArena(cap)
    live = []
    for step in range(20000):
        if live and rng.random() < 0.45:
            e = live[rng.integers(len(live))]
            if not e[2]:
                e[2] = True
                a.mark_done(e[0], e[1])
                a.release()
                live = [x for x in live if any(y[0] == x[0] and y[1] == x[1] for y in a.live)]
        else:
            n = int(rng.integers(1, 300))
            s = a.alloc(n)
            if s is not None:
                assert 0 <= s and s + n <= cap
                live.append([s, n, False])
        used = np.zeros(cap, np.int32)
        for s, n, _ in live:
            used[s:s + n] += 1
        assert used.max(initial=0) <= 1, f"overlap at step {step}"
        assert sum(n for _, n, _ in live) <= a.in_use() <= cap


# ---- scheduler with a host executor ------------------------------------------

class HostExecutor:
    """Executor on the host: an arena of numpy arrays; a batch's statistics are
    computed by the oracle from the arena contents when it is launched and
    become visible `delay` polls later."""

    def __init__(self, capacity, delay=3):
        self.src = np.zeros(capacity, np.uint32)
        self.dst = np.zeros(capacity, np.uint32)
        self.delay = delay
        self.launches = []

    def upload(self, r):
        self.src[r.start:r.start + r.n] = r.src
        self.dst[r.start:r.start + r.n] = r.dst

    def launch(self, reqs):
        first = next((r.start for r in reqs if r.n), 0)
        off = np.concatenate([[first], first + np.cumsum([r.n for r in reqs])]).astype(np.int64)
        self.launches.append([(r.rid, r.start, r.n) for r in reqs])
        out = oracle.window_stats(self.src, self.dst, off)
        return {"out": out, "polls": 0}

    def poll(self, h):
        h["polls"] += 1
        return h["polls"] > self.delay

    def results(self, h):
        return h["out"]


class FakeClock:
    def __init__(self, dt=1e-6):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        self.t += self.dt
        return self.t


def make_requests(n, lo_log2, hi_log2, seed, empty_every=0):
    wl = synth.serving_stream(seed=seed, num_windows=n, lo_log2=lo_log2, hi_log2=hi_log2)
    src, dst = wl.generate()
    off = wl.offsets
    reqs = []
    for i in range(n):
        a, b = int(off[i]), int(off[i + 1])
        if empty_every and i % empty_every == 0:
            b = a
        reqs.append(sv.Request(i, src[a:b].copy(), dst[a:b].copy()))
    return reqs


def check_exact(reqs):
    for r in reqs:
        want = oracle.window_stats(r.src, r.dst, np.array([0, r.n], np.int64))[0]
        assert np.array_equal(r.stats, want), f"request {r.rid}"


def test_closed_loop_serves_everything_exactly():
    reqs = make_requests(60, 4, 12, seed=1, empty_every=17)
    ex = HostExecutor(1 << 14)
    srv = sv.Server(ex, 1 << 14, inflight=2, clock=FakeClock())
    res = srv.run(reqs)
    assert len(res.requests) == 60
    check_exact(res.requests)
    # batches are runs of adjacent arena slots
    for launch in ex.launches:
        end = None
        for rid, start, n in launch:
            if n:
                assert end is None or start == end
                end = start + n
    assert all(r.latency > 0 for r in res.requests)
    assert srv.arena.in_use() == 0


def test_admission_waits_for_arena_space_and_wraps():
    reqs = make_requests(80, 6, 10, seed=2)
    cap = 3000                                  # a few windows at a time
    ex = HostExecutor(cap, delay=5)
    srv = sv.Server(ex, cap, inflight=2, clock=FakeClock())
    res = srv.run(reqs)
    check_exact(res.requests)
    starts = [r.start for r in res.requests if r.n]
    assert min(starts) == 0 and sum(r.n for r in reqs) > 3 * cap   # the ring wrapped
    assert max(r.admitted - r.arrival for r in res.requests) > 0     # someone waited


def test_continuous_batching_groups_arrivals_behind_a_running_batch():
    reqs = make_requests(40, 4, 8, seed=3)
    ex = HostExecutor(1 << 14, delay=50)        # a batch stays on the device a while
    srv = sv.Server(ex, 1 << 14, inflight=1, clock=FakeClock(1e-6))
    times = np.arange(40) * 5e-6                # arrivals every 5 clock ticks
    res = srv.run(reqs, arrival_times=times)
    check_exact(res.requests)
    sizes = [len(b) for b in ex.launches]
    assert sizes[0] == 1 and max(sizes) > 1     # later batches collect arrivals
    assert sum(sizes) == 40


def test_batch_limits_are_respected():
    reqs = make_requests(50, 4, 9, seed=4)
    ex = HostExecutor(1 << 15)
    srv = sv.Server(ex, 1 << 15, inflight=1, max_batch_windows=7, max_batch_packets=2000,
                    clock=FakeClock())
    res = srv.run(reqs)
    check_exact(res.requests)
    for launch in ex.launches:
        assert len(launch) <= 7
        assert sum(n for _, _, n in launch) <= max(2000, max(n for _, _, n in launch))


def test_summary_and_poisson_arrivals():
    t = sv.poisson_arrivals(20000, 1000.0, seed=9)
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 1000.0) < 40
    reqs = make_requests(30, 4, 8, seed=5)
    srv = sv.Server(HostExecutor(1 << 14), 1 << 14, clock=FakeClock())
    res = srv.run(reqs, arrival_times=np.linspace(0, 1e-4, 30))
    s = res.summary()
    assert s["windows"] == 30 and s["p99_ms"] >= s["p50_ms"] > 0
    assert s["packets"] == sum(r.n for r in reqs)


def test_oversized_window_is_rejected():
    reqs = [sv.Request(0, np.zeros(100, np.uint32), np.zeros(100, np.uint32))]
    srv = sv.Server(HostExecutor(50), 50, clock=FakeClock())
    with pytest.raises(ValueError):
        srv.run(reqs)


# ---- device executor --------------------------------------------------------------

@pytest.mark.gpu
def test_gpu_serving_each_window_alone_equals_in_mix():
    import torch

    import paper_2509_03653_amd as nsgc
    from gpu_util import assert_same, say, to_gpu

    reqs = make_requests(150, 6, 16, seed=11, empty_every=23)
    cap = 1 << 18                                # forces waits and wrap-around
    ex = sv.GpuExecutor(cap, max_batch_windows=256, streams=2)
    srv = sv.Server(ex, cap, inflight=2, max_batch_windows=256)
    say("[gpu] serving open loop")
    rate = 20000.0
    res = srv.run(reqs, arrival_times=sv.poisson_arrivals(len(reqs), rate, seed=3), timeout_s=120)
    say("[gpu] serving closed loop")
    reqs2 = make_requests(60, 6, 16, seed=12)
    res2 = srv.run(reqs2, timeout_s=120)
    for r in list(res.requests) + list(res2.requests):
        want = oracle.window_stats(r.src, r.dst, np.array([0, r.n], np.int64))
        assert_same(r.stats[None, :], want, f"served request {r.rid}")
        if r.rid % 25 == 0 and r.n:
            alone = nsgc.window_stats(to_gpu(r.src), to_gpu(r.dst), np.array([0, r.n], np.int64))
            torch.cuda.synchronize()
            assert_same(alone.cpu().numpy().view(np.uint64), r.stats[None, :], f"alone {r.rid}")
    assert res.batches < len(reqs)              # windows were batched together
    s = res.summary()
    assert s["p99_ms"] >= s["p50_ms"] > 0
