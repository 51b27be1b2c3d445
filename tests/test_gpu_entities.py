"""GPU parity of the per-entity outputs (nsgc_window_entity_counts and
nsgc_window_entities) against the oracle's sorted per-window maps.

Table III rows 3, 6 and 8 as vectors (A's non-zeros, the sources with r and
f, the destinations with c and g) and Section IV's globally unique IP count.
Lists are compared after sorting, since a window's rows come in no order.
"""
import numpy as np
import pytest

import oracle
import synth
from conftest import load_golden_batch, load_golden_windows
from gpu_util import say, to_gpu
from hashed_addresses import DESTINATION_MARKER, SOURCE_MARKER

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _default_tuning():
    import paper_2509_03653_amd as nsgc
    nsgc.set_tune(nsgc.default_tune())
    yield
    nsgc.set_tune(nsgc.default_tune())


def _sorted_rows(a):
    a = np.asarray(a, dtype=np.int64).reshape(-1, 3)
    return a[np.lexsort(a.T[::-1])] if len(a) else a


def expected(src, dst, off):
    """Oracle lists and counts per window."""
    out = []
    for w in range(len(off) - 1):
        a, b = int(off[w]), int(off[w + 1])
        e = oracle.window_entities(src, dst, a, b)
        k = e["link_keys"].astype(np.int64)
        links = np.stack([(e["link_keys"] >> np.uint64(32)).astype(np.int64),
                          (e["link_keys"] & np.uint64(0xFFFFFFFF)).astype(np.int64),
                          e["link_counts"].astype(np.int64)], 1) if k.size else np.zeros((0, 3), np.int64)
        rows = np.stack([e["row_ids"].astype(np.int64), e["row_packets"].astype(np.int64),
                         e["row_links"].astype(np.int64)], 1) if e["row_ids"].size else np.zeros((0, 3), np.int64)
        cols = np.stack([e["col_ids"].astype(np.int64), e["col_packets"].astype(np.int64),
                         e["col_links"].astype(np.int64)], 1) if e["col_ids"].size else np.zeros((0, 3), np.int64)
        out.append({"links": _sorted_rows(links), "sources": _sorted_rows(rows),
                    "destinations": _sorted_rows(cols),
                    "counts": [len(links), len(rows), len(cols), e["unique_ips"]]})
    return out


def check_entities(src, dst, off, what):
    import paper_2509_03653_amd as nsgc
    import torch
    off = np.asarray(off, np.int64)
    want = expected(src, dst, off)
    say(f"[gpu] entities {what}: windows={len(off) - 1} packets={int(off[-1] - off[0])}")
    s, d = to_gpu(src), to_gpu(dst)
    counts = nsgc.window_entity_counts(s, d, off)
    got = nsgc.window_entities(s, d, off)
    torch.cuda.synchronize()
    c1 = counts.cpu().numpy()
    c2 = got["counts"].cpu().numpy()
    lists = {k: got[k].cpu().numpy() for k in ("links", "sources", "destinations")}
    for w, e in enumerate(want):
        assert list(c1[w]) == e["counts"], (what, w, c1[w], e["counts"])
        assert list(c2[w]) == e["counts"], (what, w, c2[w], e["counts"])
        for k in ("links", "sources", "destinations"):
            o = got[{"links": "link_offsets", "sources": "source_offsets",
                     "destinations": "destination_offsets"}[k]]
            rows = _sorted_rows(lists[k][o[w]:o[w + 1]])
            np.testing.assert_array_equal(rows, e[k], err_msg=f"{what} window {w} {k}")


def test_golden_windows_and_batch():
    for name, (s, d, _) in sorted(load_golden_windows().items()):
        check_entities(s, d, np.array([0, s.size], np.int64), f"golden {name}")
    src, dst, off, _ = load_golden_batch()
    check_entities(src, dst, off, "golden batch")


def test_tiny_alphabets_extreme_and_marker_addresses():
    rng = np.random.default_rng(31)
    sizes = [0, 1, 5, 64, 700, 1024, 1025, 3000, 20000]
    off = synth.offsets_from_sizes(sizes)
    n = int(off[-1])
    alphabet = np.array([0, 1, 2, 0xFFFFFFFF, SOURCE_MARKER, DESTINATION_MARKER, 77], np.uint32)
    src = alphabet[rng.integers(0, alphabet.size, n)]
    dst = alphabet[rng.integers(0, alphabet.size, n)]
    dst[::5] = src[::5]                     # self-loops
    check_entities(src, dst, off, "tiny alphabet")


def test_mixed_window_sizes_every_path():
    # small (LDS-only), wavefront phase-B and workgroup phase-B windows
    sizes = [900, 5000, 300000, 70000, 1 << 19, 0, 2000]
    off = synth.offsets_from_sizes(sizes)
    wl = synth.zipf_batch(seed=5, num_windows=1, log2_window=4)
    src, dst = synth.fill(off, 14, wl.src_dist, wl.dst_dist)
    check_entities(src, dst, off, "mixed sizes")


def test_benchmark_batch_every_list():
    wl = synth.zipf_batch(seed=1)
    src, dst = wl.generate()
    check_entities(src, dst, wl.offsets, "64 x 2^17 Zipf")


def test_short_ranges_write_no_more_than_asked():
    import paper_2509_03653_amd as nsgc
    import torch
    wl = synth.zipf_batch(seed=2, num_windows=3, log2_window=13)
    src, dst = wl.generate()
    off = wl.offsets
    s, d = to_gpu(src), to_gpu(dst)
    counts = nsgc.window_entity_counts(s, d, off)
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    # window 1 gets half its rows in every list; the rows after it stay untouched
    caps = c[:, :3].copy()
    caps[1] //= 2
    offs = [np.concatenate([[0], np.cumsum(caps[:, k])]).astype(np.int64) for k in range(3)]
    lists = [torch.full((int(o[-1]) + 7, 3), -5, dtype=torch.int64, device="cuda") for o in offs]
    cnt = torch.empty_like(counts)
    import ctypes
    rc = nsgc.library().nsgc_window_entities(
        ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(d.data_ptr()),
        ctypes.c_void_p(off.ctypes.data), 3,
        ctypes.c_void_p(offs[0].ctypes.data), ctypes.c_void_p(lists[0].data_ptr()),
        ctypes.c_void_p(offs[1].ctypes.data), ctypes.c_void_p(lists[1].data_ptr()),
        ctypes.c_void_p(offs[2].ctypes.data), ctypes.c_void_p(lists[2].data_ptr()),
        ctypes.c_void_p(cnt.data_ptr()),
        ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream)))
    assert rc == 0
    torch.cuda.synchronize()
    np.testing.assert_array_equal(cnt.cpu().numpy(), c)
    want = expected(src, dst, off)
    for k, name in enumerate(("links", "sources", "destinations")):
        host = lists[k].cpu().numpy()
        assert (host[int(offs[k][-1]):] == -5).all(), name        # nothing past the end
        for w in (0, 2):                                         # full windows are exact
            np.testing.assert_array_equal(_sorted_rows(host[offs[k][w]:offs[k][w + 1]]), want[w][name])
        part = host[offs[k][1]:offs[k][2]]                       # the short one: a subset
        assert (part != -5).all()
        full = {tuple(r) for r in want[1][name]}
        assert all(tuple(r) in full for r in part), name
