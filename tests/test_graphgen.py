"""Seeded input generators (CPU): the batch of small graphs."""
import numpy as np

from paper_1911_10616_amd import graphgen as gg


def test_batch_small_structure():
    vptr, rp, ci = gg.batch_small(300, 11, nmin=10, nmax=60)
    n = len(rp) - 1
    assert vptr[0] == 0 and vptr[-1] == n and np.all(np.diff(vptr.astype(np.int64)) >= 10)
    src = np.repeat(np.arange(n), np.diff(rp))
    g_of = np.searchsorted(vptr, np.arange(n), side="right") - 1
    assert np.array_equal(g_of[src], g_of[ci])  # no edge joins two graphs
    deg = np.diff(rp)
    for g in range(1, 300, 2):  # Barabasi-Albert: star on 4 vertices + 3 edges per new vertex
        a, b = int(vptr[g]), int(vptr[g + 1])
        assert deg[a:b].sum() // 2 == 3 + 3 * (b - a - 4)
    er = [deg[int(vptr[g]):int(vptr[g + 1])].mean() for g in range(0, 300, 2)]
    assert 5.0 < np.mean(er) < 7.0  # mean degree 6


def test_batch_small_is_seeded():
    a = gg.batch_small(20, 5)
    b = gg.batch_small(20, 5)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
