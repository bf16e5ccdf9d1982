"""Independent brute force for tiny graphs (tests only).

A second, separately written transcription of the paper's patterns
(Fig. node_orbits: edges on 1-based node ids, and the printed orbit label of
one node per orbit), orbit classes derived by brute-force automorphisms, and
classification of every k-subset (k = 2..5) of a tiny graph by trying every
bijection onto every pattern.  No code is shared with the C oracle.
"""
from itertools import combinations, permutations

import numpy as np

# (edges, {node: label}) for H0..H29
PATTERNS = [
    ("12", {2: 0}),
    ("12 23", {2: 2, 3: 1}),
    ("12 13 23", {3: 3}),
    ("12 23 34", {3: 5, 4: 4}),
    ("13 23 34", {3: 7, 4: 6}),
    ("12 13 24 34", {3: 8}),
    ("12 23 24 34", {1: 9, 2: 11, 3: 10}),
    ("12 13 14 24 34", {2: 12, 4: 13}),
    ("12 13 14 23 24 34", {4: 14}),
    ("12 23 34 45", {3: 17, 4: 16, 5: 15}),
    ("13 23 34 45", {1: 19, 3: 21, 4: 20, 5: 18}),
    ("13 23 34 35", {3: 23, 5: 22}),
    ("13 24 34 35 45", {1: 24, 3: 26, 5: 25}),
    ("12 13 23 34 45", {1: 29, 3: 30, 4: 28, 5: 27}),
    ("13 23 34 35 45", {1: 31, 3: 33, 4: 32}),
    ("12 13 24 35 45", {5: 34}),
    ("12 23 24 35 45", {1: 35, 2: 38, 3: 37, 5: 36}),
    ("12 23 24 25 35 45", {1: 39, 2: 42, 3: 40, 5: 41}),
    ("12 13 23 34 35 45", {3: 44, 4: 43}),
    ("12 23 24 34 35 45", {1: 45, 2: 47, 3: 48, 5: 46}),
    ("12 13 14 25 35 45", {1: 50, 2: 49}),
    ("12 13 24 34 35 45", {1: 51, 3: 53, 5: 52}),
    ("13 14 23 24 34 35 45", {1: 54, 3: 55}),
    ("12 23 24 25 34 35 45", {1: 56, 2: 58, 3: 57}),
    ("12 13 23 24 34 35 45", {1: 59, 2: 60, 3: 61}),
    ("12 13 14 25 34 35 45", {2: 62, 3: 64, 5: 63}),
    ("12 13 23 24 25 34 35 45", {1: 65, 3: 67, 5: 66}),
    ("12 13 14 23 25 34 35 45", {3: 69, 4: 68}),
    ("12 13 14 23 24 25 34 35 45", {1: 70, 4: 71}),
    ("12 13 14 15 23 24 25 34 35 45", {5: 72}),
]


def _pattern(i):
    es, lab = PATTERNS[i]
    edges = [(int(t[0]) - 1, int(t[1]) - 1) for t in es.split()]
    k = 1 + max(max(e) for e in edges)
    return k, edges, {a - 1: b for a, b in lab.items()}


def _eset(edges):
    return frozenset(frozenset(e) for e in edges)


def pattern_orbits():
    """list of (k, edge set, orbit label per node)."""
    out = []
    for i in range(len(PATTERNS)):
        k, edges, lab = _pattern(i)
        es = _eset(edges)
        autos = [p for p in permutations(range(k))
                 if _eset((p[a], p[b]) for a, b in edges) == es]
        orbit = [None] * k
        for x in range(k):
            cls = {p[x] for p in autos}
            labels = {lab[y] for y in cls if y in lab}
            assert len(labels) == 1, (i, x, labels)
            orbit[x] = labels.pop()
        out.append((k, es, orbit, len(autos)))
    return out


_PO = None


def _po():
    global _PO
    if _PO is None:
        _PO = pattern_orbits()
    return _PO


_CACHE = {}


def _classify(k, es_local):
    """(pattern index, orbit per local position) of a connected k-vertex
    graph given as a set of frozenset pairs on 0..k-1."""
    key = (k, es_local)
    if key not in _CACHE:
        _CACHE[key] = _classify_uncached(k, es_local)
    return _CACHE[key]


def _classify_uncached(k, es_local):
    for h, (kk, es, orbit, _) in enumerate(_po()):
        if kk != k or len(es) != len(es_local):
            continue
        for p in permutations(range(k)):  # p: pattern node -> local position
            if _eset((p[a], p[b]) for a, b in (tuple(e) for e in es)) == es_local:
                res = [None] * k
                for x in range(k):
                    res[p[x]] = orbit[x]
                return h, res
    return None, None


def _connected(k, es):
    seen = {0}
    stack = [0]
    while stack:
        x = stack.pop()
        for e in es:
            if x in e:
                (y,) = e - {x}
                if y not in seen:
                    seen.add(y)
                    stack.append(y)
    return len(seen) == k


def adjacency_sets(row_ptr, col_idx):
    n = len(row_ptr) - 1
    return [set(int(c) for c in col_idx[row_ptr[v]:row_ptr[v + 1]]) for v in range(n)]


def induced(row_ptr, col_idx, kmax=5):
    adj = adjacency_sets(row_ptr, col_idx)
    n = len(adj)
    out = np.zeros((n, 73), np.int64)
    for k in range(2, kmax + 1):
        for S in combinations(range(n), k):
            es = _eset((i, j) for i in range(k) for j in range(i + 1, k) if S[j] in adj[S[i]])
            if not _connected(k, es):
                continue
            h, orb = _classify(k, es)
            for i in range(k):
                out[S[i], orb[i]] += 1
    return out


def noninduced(row_ptr, col_idx, kmax=5):
    """DM(u, theta): distinct non-induced copies = (vertex set, edge subset)
    pairs forming a connected spanning subgraph isomorphic to the pattern."""
    adj = adjacency_sets(row_ptr, col_idx)
    n = len(adj)
    out = np.zeros((n, 73), np.int64)
    for k in range(2, kmax + 1):
        for S in combinations(range(n), k):
            es = [frozenset((i, j)) for i in range(k) for j in range(i + 1, k) if S[j] in adj[S[i]]]
            for r in range(k - 1, len(es) + 1):
                for sub in combinations(es, r):
                    sub = frozenset(sub)
                    if not _connected(k, sub):
                        continue
                    h, orb = _classify(k, sub)
                    for i in range(k):
                        out[S[i], orb[i]] += 1
    return out


# Edge orbits of the 3- and 4-vertex patterns (Fig. edge_orbits): the
# printed label of each edge orbit and one edge of it (pattern index into
# PATTERNS, 1-based node ids of that figure).  Classes follow from brute-force
# automorphisms of the pattern's edge set.
EDGE_LABELS = [(1, (2, 3)), (2, (1, 3)), (3, (3, 4)), (3, (2, 3)), (4, (3, 4)), (5, (3, 4)),
               (6, (1, 2)), (6, (3, 4)), (6, (2, 4)), (7, (2, 4)), (7, (1, 4)), (8, (1, 4))]


def edge_orbit_classes():
    """{pattern h: (k, edges, {frozenset edge: label}, orbit per node)}."""
    po = pattern_orbits()
    out = {}
    for h in range(1, 9):
        k, es, orb, _ = po[h]
        edges = sorted(tuple(sorted(e)) for e in es)
        auts = [p for p in permutations(range(k))
                if _eset((p[a], p[b]) for a, b in edges) == es]
        label = {}
        for lab, (hh, (a, b)) in enumerate(EDGE_LABELS):
            if hh != h:
                continue
            rep = (a - 1, b - 1)
            for p in auts:
                label[frozenset((p[rep[0]], p[rep[1]]))] = lab
        assert set(label) == set(es), h
        out[h] = (k, edges, label, orb)
    return out


def edge_orbit_counts(row_ptr, col_idx):
    """int64[2m, 12]: E_i<u,v> at slot (u, v) from injective maps of every
    3- and 4-vertex pattern into the graph (edges preserved), divided by the
    pattern's automorphism count; u is the endpoint in the orbit of larger
    index, and both slots count when the endpoint orbits are equal."""
    adj = adjacency_sets(row_ptr, col_idx)
    n = len(adj)
    rp = [int(x) for x in row_ptr]
    slot = {}
    for u in range(n):
        for i, v in enumerate(int(c) for c in col_idx[rp[u]:rp[u + 1]]):
            slot[(u, v)] = rp[u] + i
    out = np.zeros((rp[-1], 12), np.int64)
    for h, (k, edges, label, orb) in edge_orbit_classes().items():
        es = _eset(edges)
        aut = sum(1 for p in permutations(range(k)) if _eset((p[a], p[b]) for a, b in edges) == es)
        acc = np.zeros_like(out)
        for f in permutations(range(n), k):
            if not all(f[b] in adj[f[a]] for a, b in edges):
                continue
            for a, b in edges:
                lab = label[frozenset((a, b))]
                if orb[a] >= orb[b]:
                    acc[slot[(f[a], f[b])], lab] += 1
                if orb[b] >= orb[a]:
                    acc[slot[(f[b], f[a])], lab] += 1
        assert (acc % aut == 0).all()
        out += acc // aut
    return out
