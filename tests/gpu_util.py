"""Helpers shared by the GPU tests: move numpy packets to the GPU and back."""
import sys

import numpy as np


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_gpu(a):
    import torch
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32)).cuda()


def gpu_stats(src, dst, offsets, form="batched", graph=None):
    import torch
    import paper_2509_03653_amd as nsgc
    s, d = to_gpu(src), to_gpu(dst)
    off = np.asarray(offsets, dtype=np.int64)
    if form == "batched":
        out = nsgc.window_stats(s, d, off)
    elif form == "plain":
        out = nsgc.window_stats_plain(s, d, off)
    elif form == "noalloc":
        out = nsgc.window_stats_noalloc(s, d, off)
    elif form == "graph":
        g = graph or nsgc.Graph(max(int(off[-1] - off[0]), 1), max(len(off) - 1, 1))
        out = g.launch(s, d, off)
        torch.cuda.synchronize()
        if graph is None:
            g.close()
    else:
        raise ValueError(form)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64)


def assert_same(got, want, what=""):
    got = np.asarray(got, dtype=np.uint64)
    want = np.asarray(want, dtype=np.uint64)
    assert got.shape == want.shape, (got.shape, want.shape, what)
    bad = np.argwhere(got != want)
    if bad.size:
        w = int(bad[0][0])
        raise AssertionError(f"{what}: {len(np.unique(bad[:, 0]))} windows differ; first w={w}\n"
                             f"gpu    {got[w].tolist()}\noracle {want[w].tolist()}")
