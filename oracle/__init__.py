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
  transform_matrix    pinned against Fig. A (with the row-5 erratum)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

NORB = 73
NGRAPHLET = 30
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orbit_oracle.c")
_LIB = os.path.join(_HERE, "liborbit_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over roots)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-fopenmp", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
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
