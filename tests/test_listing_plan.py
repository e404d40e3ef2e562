"""Host logic of chunked listing: greedy cut points over per-rank counts."""
import numpy as np
import pytest

from paper_2311_13798_amd.listing import cuts_from_counts


def brute_cuts(counts, cap):
    cuts, i, m = [0], 0, len(counts)
    while i < m:
        j, s = i, 0
        while j < m and s + counts[j] <= cap:
            s += counts[j]
            j += 1
        if j == i:
            raise ValueError
        cuts.append(j)
        i = j
    return cuts


@pytest.mark.parametrize("seed", range(20))
def test_cuts_match_a_greedy_scan(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 300))
    counts = rng.integers(0, 50, size=m) * (rng.random(m) < 0.7)
    cap = int(max(counts.max(initial=0), 1) * rng.integers(1, 6))
    cuts, sizes = cuts_from_counts(counts.astype(np.uint64), cap)
    assert cuts == brute_cuts(list(map(int, counts)), cap)
    assert sizes == [int(counts[a:b].sum()) for a, b in zip(cuts[:-1], cuts[1:])]
    assert all(s <= cap for s in sizes) and sum(sizes) == int(counts.sum())


def test_a_seed_larger_than_the_buffer_is_an_error():
    with pytest.raises(ValueError):
        cuts_from_counts(np.array([1, 10, 1], np.uint64), 5)


def test_counts_beyond_int64():
    counts = np.array([2 ** 62, 2 ** 62, 2 ** 62, 5], np.uint64)
    cuts, sizes = cuts_from_counts(counts, 2 ** 63)
    assert cuts == [0, 2, 4] and sizes == [2 ** 63, 2 ** 62 + 5]
