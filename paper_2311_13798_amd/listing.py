"""Listing every k-clique of a graph whose listing exceeds one device buffer: rank-range chunks.

Every k-clique is listed exactly once, under its seed edge (the first of its edges in the truss-based
edge order, Section 4.1), so ranges of seed ranks partition the listing.  Chunk cut points come from
per-seed counts; the order-independent checksums of the chunks add up (mod 2^64) to that of the whole
listing.
"""
from __future__ import annotations

import numpy as np

from . import ARR_RANK, ebbkc_count_seeds, ebbkc_list


def cuts_from_counts(by_rank, cap: int):
    """Greedy cut points 0 = r_0 < ... < r_c = m over per-rank counts so that every chunk holds at
    most cap items (each chunk as long as it can be); returns (cuts, per-chunk totals)."""
    m = len(by_rank)
    cum = np.cumsum(np.asarray(by_rank, dtype=np.uint64), dtype=np.uint64)
    cuts, sizes, base = [0], [], 0
    while cuts[-1] < m:
        r = int(np.searchsorted(cum, np.uint64(min(base + cap, (1 << 64) - 1)), side="right"))
        if r <= cuts[-1]:
            raise ValueError(f"the item at rank {cuts[-1]} alone is larger than the chunk capacity {cap}")
        r = min(r, m)
        sizes.append(int(cum[r - 1]) - base)
        base = int(cum[r - 1])
        cuts.append(r)
    return cuts, sizes


def plan_chunks(G, k: int, cap: int):
    """Cut points of the seed ranks of G such that every chunk holds at most cap k-cliques (per-seed
    counts from the library); returns (cuts, per-chunk counts)."""
    m = int(G.info.m)
    per = np.zeros(m, np.uint64)
    ebbkc_count_seeds(G.handle, k, np.arange(m, dtype=np.int64), per)
    by_rank = np.empty(m, np.uint64)
    by_rank[G.export(ARR_RANK)] = per
    return cuts_from_counts(by_rank, cap)


def list_in_chunks(G, k: int, buf, cap: int, flags: int = 0, cuts=None, on_chunk=None):
    """List every k-clique of G chunk by chunk into buf (device, at least cap x k int32).  on_chunk(a, b,
    written) is called after each chunk, while its tuples are in buf.  Returns (total, unordered
    checksum of the whole listing, number of chunks)."""
    if cuts is None:
        cuts, _ = plan_chunks(G, k, cap)
    total, hu = 0, 0
    for a, b in zip(cuts[:-1], cuts[1:]):
        w, _, u = ebbkc_list(G.handle, k, buf, cap, flags, a, b)
        total += w
        hu = (hu + u) % (1 << 64)
        if on_chunk:
            on_chunk(a, b, w)
    return total, hu, len(cuts) - 1
