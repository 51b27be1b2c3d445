"""Independent formulations used to pin the oracle (not used by the HIP path).

Both compute the nine statistics of Table III (and its src/dst reverse) for
one window, by routes that share nothing with the oracle's ordered maps:

* ``brute_force`` -- O(n^2) pairwise equality matrices, no maps or sorting.
  Packet i opens a new link if no earlier packet has the same (src, dst);
  a source's fan-out counts the link-opening packets it sent.
* ``numpy_unique`` -- the sort-based formulation: ``numpy.unique`` on packed
  keys with counts gives A's non-zeros; a second ``numpy.unique`` on the
  link rows / columns gives the per-source and per-destination totals.
"""
from __future__ import annotations

import numpy as np


def brute_force(src, dst) -> np.ndarray:
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    n = src.size
    if n == 0:
        return np.zeros(9, dtype=np.uint64)
    eq_s = src[:, None] == src[None, :]
    eq_d = dst[:, None] == dst[None, :]
    eq_p = eq_s & eq_d
    strictly_earlier = np.tril(np.ones((n, n), dtype=bool), -1)   # [i, j] : j < i
    opens_link = ~np.any(eq_p & strictly_earlier, axis=1)          # first packet of its pair
    first_src = ~np.any(eq_s & strictly_earlier, axis=1)
    first_dst = ~np.any(eq_d & strictly_earlier, axis=1)
    multiplicity = eq_p.sum(axis=1)                                # A(s_i, d_i)
    r = eq_s.sum(axis=1)                                           # r(s_i)
    c = eq_d.sum(axis=1)                                           # c(d_i)
    f = (eq_s & opens_link[None, :]).sum(axis=1)                   # f(s_i)
    g = (eq_d & opens_link[None, :]).sum(axis=1)                   # g(d_i)
    valid = int(multiplicity[opens_link].sum())
    return np.array([
        valid, int(opens_link.sum()), int(multiplicity.max()),
        int(first_src.sum()), int(r.max()), int(f.max()),
        int(first_dst.sum()), int(c.max()), int(g.max()),
    ], dtype=np.uint64)


def numpy_unique(src, dst) -> np.ndarray:
    src = np.asarray(src, dtype=np.uint64)
    dst = np.asarray(dst, dtype=np.uint64)
    if src.size == 0:
        return np.zeros(9, dtype=np.uint64)
    keys = (src << np.uint64(32)) | dst
    links, counts = np.unique(keys, return_counts=True)
    counts = counts.astype(np.int64)
    link_src = links >> np.uint64(32)
    link_dst = links & np.uint64(0xFFFFFFFF)

    def grouped(ids):
        uniq, inv = np.unique(ids, return_inverse=True)
        packets = np.zeros(uniq.size, dtype=np.int64)
        np.add.at(packets, inv, counts)
        fan = np.bincount(inv, minlength=uniq.size).astype(np.int64)
        return uniq.size, int(packets.max()), int(fan.max())

    ns, rmax, fmax = grouped(link_src)
    nd, cmax, gmax = grouped(link_dst)
    return np.array([int(counts.sum()), links.size, int(counts.max()), ns, rmax, fmax,
                     nd, cmax, gmax], dtype=np.uint64)


def brute_force_unique_ips(src, dst) -> int:
    """|{src} U {dst}| by pairwise comparison: an address counts where it
    first occurs in the sequence src[0], dst[0], src[1], dst[1], ..."""
    seq = np.empty(2 * len(src), dtype=np.int64)
    seq[0::2] = np.asarray(src, dtype=np.int64)
    seq[1::2] = np.asarray(dst, dtype=np.int64)
    n = seq.size
    if n == 0:
        return 0
    eq = seq[:, None] == seq[None, :]
    earlier = np.tril(np.ones((n, n), dtype=bool), -1)
    return int((~np.any(eq & earlier, axis=1)).sum())
