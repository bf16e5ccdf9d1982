"""CPU oracle for per-vertex graphlet orbit counts -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.

It wraps ``orbit_oracle.c`` (plain C, built with gcc by :func:`build`), which
counts orbits by visiting every connected induced subset of 2..5 vertices and
classifying it with a table generated from the paper's figure of all vertex
orbits (Fig. node_orbits) by computing automorphisms.

Parity status of each function (what pins it is listed in the tests):
  induced_counts      pinned (closed forms, invariants, brute force, paper's
                      orbit-26 equation and Fig. A via noninduced_counts)
  noninduced_counts   pinned (paper's 4-vertex lemma equations, eq. orb26,
                      brute-force injective maps, Fig. A)
  rooted_counts       pinned against induced_counts (same definition)
  edge_counts         pinned (Lemma 4edgeorbit equations on brute-force T, C4,
                      K4; brute-force injective maps; closed forms)
  transform_matrix    pinned against Fig. A (with the row-5 erratum)
  overflow_flags      the overflow reading of integer width (the paper is
                      silent on it): pinned by brute-force homomorphism
                      counts of every rooted tree shape on tiny graphs and by
                      the bound holding over every non-induced count
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

NORB = 73
NGRAPHLET = 30
NEORB = 12
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orbit_oracle.c")
_LIB = os.path.join(_HERE, "liborbit_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over roots)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-fopenmp", "-pthread", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_tables_status.restype = ctypes.c_int
        lib.oracle_tables.argtypes = [ip, ip, ip, ip, ip]
        lib.oracle_classify_mask.argtypes = [ctypes.c_int, ctypes.c_int, ip]
        lib.oracle_classify_mask.restype = ctypes.c_int
        lib.oracle_pair_index.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.oracle_pair_index.restype = ctypes.c_int
        for f in (lib.oracle_induced_counts, lib.oracle_noninduced_counts):
            f.argtypes = [u32p, u32p, ctypes.c_uint32, ctypes.c_int, u64p, ctypes.c_int]
            f.restype = ctypes.c_int
        lib.oracle_rooted_counts.argtypes = [u32p, u32p, ctypes.c_uint32, ctypes.c_int, u32p,
                                             ctypes.c_uint32, ctypes.c_uint64, u64p,
                                             ctypes.POINTER(ctypes.c_uint8), ctypes.c_int]
        lib.oracle_rooted_counts.restype = ctypes.c_int
        lib.oracle_edge_counts.argtypes = [u32p, u32p, ctypes.c_uint32, u64p, ctypes.c_int]
        lib.oracle_edge_counts.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _graph(row_ptr, col_idx):
    rp = np.ascontiguousarray(row_ptr, dtype=np.uint32)
    ci = np.ascontiguousarray(col_idx, dtype=np.uint32)
    if ci.size == 0:
        ci = np.zeros(1, np.uint32)
    return rp, ci, len(rp) - 1


def tables_status() -> int:
    return _load().oracle_tables_status()


def tables():
    """Pattern tables derived from the figure by computing automorphisms.

    Returns dict with node_orbit[30,5] (-1 past k), aut[30], orbit_graphlet[73],
    orbit_size[73], pattern_k[30]."""
    lib = _load()
    no = np.zeros(NGRAPHLET * 5, np.int32)
    aut = np.zeros(NGRAPHLET, np.int32)
    og = np.zeros(NORB, np.int32)
    osz = np.zeros(NORB, np.int32)
    pk = np.zeros(NGRAPHLET, np.int32)
    ip = ctypes.c_int
    lib.oracle_tables(_ptr(no, ip), _ptr(aut, ip), _ptr(og, ip), _ptr(osz, ip), _ptr(pk, ip))
    return {"node_orbit": no.reshape(NGRAPHLET, 5), "aut": aut, "orbit_graphlet": og,
            "orbit_size": osz, "pattern_k": pk}


def classify_mask(k: int, mask: int):
    """(graphlet id or -1, orbit of each of the k positions) of a labelled mask."""
    out = np.zeros(5, np.int32)
    g = _load().oracle_classify_mask(k, mask, _ptr(out, ctypes.c_int))
    return g, out[:k].copy()


def pair_index(i: int, j: int) -> int:
    return _load().oracle_pair_index(i, j)


def induced_counts(row_ptr, col_idx, kmax: int = 5, threads: int = 1) -> np.ndarray:
    """uint64[n, 73]: induced orbit counts (orbits of patterns with > kmax
    vertices are zero)."""
    rp, ci, n = _graph(row_ptr, col_idx)
    out = np.zeros((max(n, 1), NORB), np.uint64)
    rc = _load().oracle_induced_counts(_ptr(rp, ctypes.c_uint32), _ptr(ci, ctypes.c_uint32), n,
                                       kmax, _ptr(out, ctypes.c_uint64), threads)
    if rc:
        raise RuntimeError(f"oracle failed: {rc}")
    return out[:n]


def noninduced_counts(row_ptr, col_idx, kmax: int = 5, threads: int = 1) -> np.ndarray:
    """uint64[n, 73]: non-induced orbit counts DM(u, theta)."""
    rp, ci, n = _graph(row_ptr, col_idx)
    out = np.zeros((max(n, 1), NORB), np.uint64)
    rc = _load().oracle_noninduced_counts(_ptr(rp, ctypes.c_uint32), _ptr(ci, ctypes.c_uint32),
                                          n, kmax, _ptr(out, ctypes.c_uint64), threads)
    if rc:
        raise RuntimeError(f"oracle failed: {rc}")
    return out[:n]


def edge_counts(row_ptr, col_idx, threads: int = 1) -> np.ndarray:
    """uint64[2m, 12]: non-induced edge orbit counts E_0..E_11 of every CSR
    slot (u, v) -- for an edge orbit whose two endpoint vertex orbits
    differ, the count with u in the endpoint orbit of larger index
    (Definition edge-orbit; matches as defined after Fig. edge_orbits)."""
    rp, ci, n = _graph(row_ptr, col_idx)
    m2 = int(rp[-1]) if n >= 0 else 0
    out = np.zeros((max(m2, 1), NEORB), np.uint64)
    rc = _load().oracle_edge_counts(_ptr(rp, ctypes.c_uint32), _ptr(ci, ctypes.c_uint32), n,
                                    _ptr(out, ctypes.c_uint64), threads)
    if rc:
        raise RuntimeError(f"oracle failed: {rc}")
    return out[:m2]


def rooted_counts(row_ptr, col_idx, roots, kmax: int = 5, budget: int = 0, threads: int = 1):
    """(uint64[len(roots), 73], bool[len(roots)] complete) for the listed roots."""
    rp, ci, n = _graph(row_ptr, col_idx)
    roots = np.ascontiguousarray(roots, dtype=np.uint32)
    nr = roots.size
    out = np.zeros((max(nr, 1), NORB), np.uint64)
    comp = np.zeros(max(nr, 1), np.uint8)
    rc = _load().oracle_rooted_counts(_ptr(rp, ctypes.c_uint32), _ptr(ci, ctypes.c_uint32), n,
                                      kmax, _ptr(roots if nr else np.zeros(1, np.uint32),
                                                 ctypes.c_uint32),
                                      nr, budget, _ptr(out, ctypes.c_uint64),
                                      _ptr(comp, ctypes.c_uint8), threads)
    if rc:
        raise RuntimeError(f"oracle failed: {rc}")
    return out[:nr], comp[:nr].astype(bool)


def transform_matrix() -> np.ndarray:
    """A (73 x 73, int64): A[i, j] = non-induced count of orbit i at a vertex
    of orbit j, computed with pattern H(j) itself as the input graph (section
    on conversion between induced and non-induced counts).  Block-diagonal
    by pattern size; induced -> non-induced is N = A I."""
    t = tables()
    A = np.zeros((NORB, NORB), np.int64)
    for h in range(NGRAPHLET):
        k = int(t["pattern_k"][h])
        # rebuild H(h) on positions 0..k-1 from the LUT: find the mask whose
        # orbit row equals the pattern's own node orbits in node order
        want = t["node_orbit"][h][:k]
        edges = _pattern_edges(h)
        from_edges = _csr_from_pairs(k, edges)
        cnt = noninduced_counts(*from_edges, kmax=5)
        same_k = np.array([t["pattern_k"][t["orbit_graphlet"][i]] == k for i in range(NORB)])
        for x in range(k):
            A[same_k, want[x]] = cnt[x].astype(np.int64)[same_k]
    return A


def _csr_from_pairs(n, pairs):
    adj = [[] for _ in range(n)]
    for a, b in pairs:
        adj[a].append(b)
        adj[b].append(a)
    rp = np.zeros(n + 1, np.uint32)
    ci = []
    for v in range(n):
        ci.extend(sorted(adj[v]))
        rp[v + 1] = len(ci)
    return rp, np.array(ci, np.uint32)


def _pattern_edges(h):
    """Edges (0-based) of pattern h, recovered from the oracle's LUT: the
    identity labelling of the pattern is the mask whose orbit row matches."""
    t = tables()
    k = int(t["pattern_k"][h])
    want = list(t["node_orbit"][h][:k])
    # The C side keeps the transcription; recover a copy through
    # classify_mask: any mask of this pattern whose orbit row equals the
    # node-order orbits is an isomorphic copy with the same orbit
    # assignment, which is all A needs.
    for mask in range(1 << (k * (k - 1) // 2)):
        g, orb = classify_mask(k, mask)
        if g == h and list(orb) == want:
            return [(i, j) for j in range(1, k) for i in range(j)
                    if mask >> pair_index(i, j) & 1]
    raise RuntimeError("pattern not found in LUT")


# ------------------------------------------------------------ overflow flags
# The paper never discusses integer width.  Reading: counts are exact
# modulo 2^64, and a row is flagged when an upper bound of its non-induced
# counts reaches 2^63.  A non-induced copy of a connected k-vertex pattern at
# u is a connected k-vertex subgraph containing u; it holds a spanning tree,
# and at most 2^(C(k,2)-(k-1)) subgraphs of one vertex set share that tree.
# The trees with k vertices containing u number at most
# sum over rooted shapes tau of hom(tau, G; root -> u) / |Aut_root(tau)|.
ROOTED_TREES = {
    # shape name: (vertices, root-fixing automorphisms); a shape is written
    # as the tuple of its root's child subtrees
    3: [("P3_end", 1), ("P3_mid", 2)],
    4: [("P4_end", 1), ("S3_leaf", 2), ("P4_inner", 1), ("S3_centre", 6)],
    5: [("P5_end", 1), ("fork_tip", 2), ("chair_end", 1), ("S4_leaf", 6),
        ("P5_second", 1), ("fork_second", 2), ("P5_centre", 2), ("chair_deg3", 2),
        ("S4_centre", 24)],
}


def rooted_tree_homs(row_ptr, col_idx):
    """dict shape -> float64[n] of hom(tau, G; root -> u), by the nested
    neighbour sums of the degrees (child subtrees multiply, a child's count
    is summed over the neighbours it can map to)."""
    rp = np.asarray(row_ptr, np.int64)
    ci = np.asarray(col_idx, np.int64)
    n = rp.size - 1
    d = np.diff(rp).astype(np.float64)
    src = np.repeat(np.arange(n), np.diff(rp))

    def nsum(x):  # sum over neighbours
        return np.bincount(src, weights=x[ci], minlength=n) if ci.size else np.zeros(n)

    s1 = nsum(d)            # root - v - (leaf)
    q1 = nsum(d * d)        # root - v with two leaves
    c1 = nsum(d ** 3)       # root - v with three leaves
    s2 = nsum(s1)           # root - v - w - (leaf)
    q2 = nsum(q1)           # root - v - w with two leaves
    r1 = nsum(d * s1)       # root - v, v with a leaf and a 2-path
    s3 = nsum(s2)           # path of 5 from the root
    return {
        "P3_end": s1, "P3_mid": d * d,
        "P4_end": s2, "S3_leaf": q1, "P4_inner": s1 * d, "S3_centre": d ** 3,
        "P5_end": s3, "fork_tip": q2, "chair_end": r1, "S4_leaf": c1,
        "P5_second": s2 * d, "fork_second": q1 * d, "P5_centre": s1 * s1,
        "chair_deg3": s1 * d * d, "S4_centre": d ** 4,
    }


def count_bound(row_ptr, col_idx):
    """float64[n]: upper bound of every non-induced count of each vertex."""
    h = rooted_tree_homs(row_ptr, col_idx)
    d = np.diff(np.asarray(row_ptr, np.int64)).astype(np.float64)
    tot = d.copy()
    for k, extra in ((3, 2.0), (4, 8.0), (5, 64.0)):
        b = np.zeros_like(d)
        for name, aut in ROOTED_TREES[k]:
            b += h[name] / aut
        tot += extra * b
    return tot


def overflow_flags(row_ptr, col_idx) -> np.ndarray:
    """uint8[n]: 1 where the count bound reaches 2^63 (less a 1e-9 relative
    margin for the rounding of the fp64 sums)."""
    return (count_bound(row_ptr, col_idx) >= 2.0 ** 63 * (1 - 1e-9)).astype(np.uint8)
