"""Seeded synthetic graph generators and the symmetric-CSR builder.

This module holds no orbit-counting arithmetic: it only produces simple
undirected graphs (directions, duplicates and self-loops removed, as the
paper's input model in its Preliminaries section requires) in the layout
the counting library consumes:

* ``row_ptr``: uint32[n+1], ``row_ptr[n] == 2m``
* ``col_idx``: uint32[2m], each neighbour list strictly ascending.

Every generator draws from numpy's PCG64 with an explicit seed, so a
(generator, parameters, seed) triple names one graph on every platform.
It is shared by the tests, the benchmark and the CPU oracle's drivers.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "csr_from_edges", "erdos_renyi", "chung_lu", "rmat", "barabasi_albert",
    "complete", "cycle", "star", "complete_bipartite", "path", "from_edge_list",
    "random_small", "relabel", "batch_small", "CONFIG_SEED_BASE", "workload",
]

CONFIG_SEED_BASE = 0x5EED0000


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray):
    """Symmetrise, drop self-loops and duplicates, sort; return (row_ptr, col_idx)."""
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    if u.size:
        if u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n:
            raise ValueError("edge endpoint out of range")
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * np.int64(n) + hi)
    lo = key // n
    hi = key % n
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    counts = np.bincount(src, minlength=n) if src.size else np.zeros(n, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**32:
        raise ValueError("2m must fit in uint32")
    return row_ptr.astype(np.uint32), dst.astype(np.uint32)


def from_edge_list(n, edges):
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    return csr_from_edges(n, e[:, 0], e[:, 1])


def erdos_renyi(n: int, p: float, seed: int):
    """G(n, p): every unordered pair independently with probability p."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if n < 2:
        return csr_from_edges(n, [], [])
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(iu.size) < p
    return csr_from_edges(n, iu[keep], ju[keep])


def chung_lu(n: int, mean_deg: float, gamma: float, wmax: float, pairs: int, seed: int):
    """Chung-Lu power-law graph.

    Weights w_i = min(wmax, c (i+1)^(-1/(gamma-1))) with c chosen so that
    mean(w) == mean_deg; ``pairs`` endpoint pairs are drawn i.i.d. with
    probability proportional to w, then self-loops and duplicates go.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    base = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    lo_c, hi_c = 0.0, mean_deg * n
    for _ in range(200):  # bisection for the scale c
        c = 0.5 * (lo_c + hi_c)
        if np.minimum(wmax, c * base).mean() < mean_deg:
            lo_c = c
        else:
            hi_c = c
    w = np.minimum(wmax, c * base)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    out_u = np.empty(pairs, dtype=np.int64)
    out_v = np.empty(pairs, dtype=np.int64)
    chunk = 1 << 22
    for s in range(0, pairs, chunk):
        k = min(chunk, pairs - s)
        out_u[s:s + k] = np.searchsorted(cdf, rng.random(k), side="right")
        out_v[s:s + k] = np.searchsorted(cdf, rng.random(k), side="right")
    np.minimum(out_u, n - 1, out=out_u)
    np.minimum(out_v, n - 1, out=out_v)
    return csr_from_edges(n, out_u, out_v)


def rmat(scale: int, edge_factor: int, a=0.57, b=0.19, c=0.19, d=0.05, seed: int = 0,
         permute: bool = True):
    """R-MAT (Graph500 convention): edge_factor * 2^scale samples, no noise,
    seeded random vertex permutation, then symmetrise and deduplicate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 1 << scale
    ne = edge_factor * n
    u = np.zeros(ne, dtype=np.int64)
    v = np.zeros(ne, dtype=np.int64)
    ab = a + b
    c_norm = c / (c + d)
    a_norm = a / (a + b)
    chunk = 1 << 22
    for s in range(0, ne, chunk):
        k = min(chunk, ne - s)
        uu = np.zeros(k, dtype=np.int64)
        vv = np.zeros(k, dtype=np.int64)
        for bit in range(scale):
            r1 = rng.random(k)
            r2 = rng.random(k)
            ibit = r1 > ab
            jbit = np.where(ibit, r2 > c_norm, r2 > a_norm)
            uu |= ibit.astype(np.int64) << bit
            vv |= jbit.astype(np.int64) << bit
        u[s:s + k] = uu
        v[s:s + k] = vv
    if permute:
        perm = rng.permutation(n)
        u = perm[u]
        v = perm[v]
    return csr_from_edges(n, u, v)


def barabasi_albert(n: int, m_attach: int, seed: int):
    """Barabasi-Albert: a star on m_attach+1 vertices as the seed graph; each
    new vertex attaches to m_attach distinct earlier vertices chosen with
    probability proportional to degree."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m0 = m_attach + 1
    if n <= m0:
        return star(n - 1) if n >= 2 else csr_from_edges(n, [], [])
    eu = [0] * m_attach
    ev = list(range(1, m0))
    targets = eu + ev  # endpoint multiset: degree-proportional sampling
    for new in range(m0, n):
        chosen = set()
        while len(chosen) < m_attach:
            chosen.add(targets[int(rng.integers(len(targets)))])
        for t in sorted(chosen):
            eu.append(new)
            ev.append(t)
            targets.append(new)
            targets.append(t)
    return csr_from_edges(n, np.array(eu), np.array(ev))


def complete(n):
    iu, ju = np.triu_indices(n, k=1)
    return csr_from_edges(n, iu, ju)


def cycle(n):
    idx = np.arange(n)
    return csr_from_edges(n, idx, (idx + 1) % n)


def path(n):
    idx = np.arange(n - 1)
    return csr_from_edges(n, idx, idx + 1)


def star(s):
    """K_{1,s}: vertex 0 is the centre."""
    return csr_from_edges(s + 1, np.zeros(s, np.int64), np.arange(1, s + 1))


def complete_bipartite(a, b):
    """K_{a,b}: vertices 0..a-1 on one side, a..a+b-1 on the other."""
    iu, ju = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return csr_from_edges(a + b, iu.ravel(), ju.ravel())


def random_small(n: int, p: float, seed: int):
    """Small G(n,p) graph for exhaustive-style tests."""
    return erdos_renyi(n, p, seed)


def relabel(row_ptr, col_idx, seed: int):
    """The same graph with vertex ids permuted uniformly at random (vertex
    u becomes perm[u]); real graphs carry ids unrelated to degree."""
    n = len(row_ptr) - 1
    perm = np.random.Generator(np.random.PCG64(seed)).permutation(n)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr).astype(np.int64))
    keep = src < col_idx
    return csr_from_edges(n, perm[src[keep]], perm[col_idx[keep].astype(np.int64)])


def batch_small(num_graphs: int, seed: int, nmin: int = 10, nmax: int = 500,
                er_mean_deg: float = 6.0, ba_m: int = 3):
    """Many small graphs as one CSR (the disjoint union over global ids).

    Graph g has n_g ~ uniform{nmin..nmax} vertices; even g are
    Erdos-Renyi G(n_g, er_mean_deg / (n_g - 1)), odd g Barabasi-Albert with
    ba_m edges per new vertex (the model of ``barabasi_albert``: a star on
    ba_m + 1 vertices, then each new vertex draws endpoints of existing
    edges until it has ba_m distinct targets).  Returns (vptr, row_ptr,
    col_idx): graph g owns vertices vptr[g] .. vptr[g+1]-1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(nmin, nmax + 1, num_graphs).astype(np.int64)
    vptr = np.zeros(num_graphs + 1, dtype=np.int64)
    np.cumsum(sizes, out=vptr[1:])
    us, vs = [], []
    # Erdos-Renyi graphs: a binomial number of distinct pairs
    for g in range(0, num_graphs, 2):
        n = int(sizes[g])
        pairs = n * (n - 1) // 2
        k = int(rng.binomial(pairs, min(1.0, er_mean_deg / (n - 1))))
        idx = rng.choice(pairs, size=k, replace=False)
        # pair index -> (i, j), i < j, row-major over the upper triangle
        i = (n - 2 - np.floor(np.sqrt(-8.0 * idx + 4.0 * n * (n - 1) - 7) / 2.0 - 0.5)).astype(np.int64)
        j = idx + i + 1 - (n * (n - 1) // 2 - (n - i) * (n - i - 1) // 2)
        us.append(vptr[g] + i)
        vs.append(vptr[g] + j)
    # Barabasi-Albert graphs, grown in lockstep (one new vertex per graph per step)
    ba = np.arange(1, num_graphs, 2)
    if ba.size:
        m0 = ba_m + 1
        nb = sizes[ba]
        cap = 2 * (ba_m + ba_m * max(0, int(nb.max()) - m0))
        ends = np.zeros((ba.size, cap), dtype=np.int64)  # local ids of edge endpoints
        ends[:, 0:2 * ba_m:2] = 0
        ends[:, 1:2 * ba_m:2] = np.arange(1, m0)
        length = np.full(ba.size, 2 * ba_m, dtype=np.int64)
        us.append(np.repeat(vptr[ba], ba_m))
        vs.append((vptr[ba][:, None] + np.arange(1, m0)[None, :]).ravel())
        for new in range(m0, int(nb.max())):
            act = np.flatnonzero(nb > new)
            chosen = np.full((act.size, ba_m), -1, dtype=np.int64)
            for k in range(ba_m):
                todo = np.arange(act.size)
                while todo.size:
                    pick = ends[act[todo], (rng.random(todo.size) * length[act[todo]]).astype(np.int64)]
                    dup = (chosen[todo, :k] == pick[:, None]).any(axis=1)
                    chosen[todo[~dup], k] = pick[~dup]
                    todo = todo[dup]
            base = vptr[ba[act]]
            us.append(np.repeat(base + new, ba_m))
            vs.append((base[:, None] + chosen).ravel())
            rows = act
            pos = length[rows]
            ends[rows[:, None], pos[:, None] + 2 * np.arange(ba_m)[None, :]] = new
            ends[rows[:, None], pos[:, None] + 2 * np.arange(ba_m)[None, :] + 1] = chosen
            length[rows] += 2 * ba_m
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    rp, ci = csr_from_edges(int(vptr[-1]), u, v)
    return vptr.astype(np.uint64), rp, ci


def workload(name: str):
    """The five named synthetic workloads (seed = 0x5EED0000 + index)."""
    if name == "er2000":
        return erdos_renyi(2000, 0.005, CONFIG_SEED_BASE + 1)
    if name == "chunglu1m":
        return chung_lu(1_000_000, 20.0, 2.1, 50_000.0, 10_000_000, CONFIG_SEED_BASE + 2)
    if name == "chunglu1m_perm":
        return relabel(*workload("chunglu1m"), CONFIG_SEED_BASE + 6)
    if name == "chunglu250k":  # a smaller graph of the same family (cost-model training)
        return chung_lu(250_000, 20.0, 2.1, 12_500.0, 2_500_000, CONFIG_SEED_BASE + 7)
    if name == "batch100k":
        return batch_small(100_000, CONFIG_SEED_BASE + 4)
    if name == "rmat22":
        return rmat(22, 16, seed=CONFIG_SEED_BASE + 3)
    if name == "rmat24":
        return rmat(24, 32, seed=CONFIG_SEED_BASE + 5)
    raise KeyError(name)
