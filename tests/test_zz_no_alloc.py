"""GPU checks of the fixed-scratch entry point (nsgc_window_stats_noalloc):
its results equal the batched entry point's, bit for bit, on consecutive
calls of different sizes and streams; a batch beyond the fixed scratch is
refused with nothing written."""
import numpy as np
import pytest

import oracle
import paper_2509_03653_amd as nsgc
import synth
from gpu_util import assert_same, say, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _default_tune():
    nsgc.set_tune(nsgc.default_tune())
    yield
    nsgc.set_tune(nsgc.default_tune())


def _mixed_batch(seed, windows, log2_window, tiny):
    """Zipf windows of 2^log2_window packets followed by tiny windows (the
    small tier) and an empty one."""
    wl = synth.zipf_batch(seed=seed, num_windows=windows, log2_window=log2_window)
    s, d = wl.generate()
    rng = np.random.default_rng(seed)
    sizes = [int(x) for x in rng.integers(1, 1500, tiny)] + [0]
    ts = rng.integers(0, 50, sum(sizes), dtype=np.uint32)
    td = rng.integers(0, 50, sum(sizes), dtype=np.uint32)
    src = np.concatenate([s, ts]).astype(np.uint32)
    dst = np.concatenate([d, td]).astype(np.uint32)
    off = np.concatenate([np.asarray(wl.offsets, np.int64),
                          s.size + np.cumsum(sizes)]).astype(np.int64)
    return src, dst, off


def _both(src, dst, off, stream=None):
    import torch
    gs, gd = to_gpu(src), to_gpu(dst)
    w = len(off) - 1
    out_ref = torch.empty((w, 9), dtype=torch.int64, device="cuda")
    out_fix = torch.full((w, 9), -1, dtype=torch.int64, device="cuda")
    nsgc.window_stats(gs, gd, off, out=out_ref, stream=stream)
    nsgc.window_stats_noalloc(gs, gd, off, out=out_fix, stream=stream)
    torch.cuda.synchronize()
    return (out_fix.cpu().numpy().view(np.uint64), out_ref.cpu().numpy().view(np.uint64))


def test_noalloc_equals_batched_on_two_calls_second_smaller():
    import torch
    big = _mixed_batch(seed=5, windows=20, log2_window=17, tiny=30)
    small = _mixed_batch(seed=6, windows=3, log2_window=14, tiny=5)
    for name, (src, dst, off) in (("first", big), ("second, smaller", small)):
        say(f"[gpu] noalloc {name}: windows={len(off) - 1} packets={int(off[-1])}")
        got, ref = _both(src, dst, off)
        assert_same(got, ref, f"noalloc vs batched ({name})")
        want = oracle.window_stats(src, dst, off, threads=8)
        assert_same(got, want, f"noalloc vs oracle ({name})")
    # and again on another stream: the call is ordered after the previous one
    side = torch.cuda.Stream()
    src, dst, off = big
    say("[gpu] noalloc on a side stream")
    got, ref = _both(src, dst, off, stream=side)
    assert_same(got, ref, "noalloc vs batched (side stream)")


def test_noalloc_refuses_a_batch_beyond_its_scratch():
    import torch
    # one window of 6M packets needs about 24 B per packet of workspace
    n = 6 << 20
    off = np.array([0, n], np.int64)
    sizes = nsgc.plan_sizes(off)
    assert sizes["workspace_bytes"] > nsgc.NOALLOC_SCRATCH_BYTES - nsgc.NOALLOC_PLAN_BYTES
    s = torch.zeros(n, dtype=torch.int32, device="cuda")
    out = torch.full((1, 9), -1, dtype=torch.int64, device="cuda")
    say("[gpu] noalloc oversize batch")
    with pytest.raises(nsgc.NsgcError) as e:
        nsgc.window_stats_noalloc(s, s, off, out=out)
    assert e.value.status == -7
    torch.cuda.synchronize()
    assert (out.cpu() == -1).all()
