"""Generate ``csrc/orbit_tables.h``: the non-induced -> induced transform.

Section "Conversion between Induced and Noninduced counts" of the paper:
for every vertex the non-induced orbit counts N and induced counts I are
related by N = A I, with A[i, j] the number of non-induced copies of orbit
i that one induced copy of orbit j contains, at a vertex of orbit j.  A is
block-diagonal by pattern size (a non-induced k-vertex copy lives in one
induced k-vertex subset).  The paper prints only the 4-vertex block (Fig. A)
and points elsewhere for the 5-vertex one, so this script derives every
block from the pattern definitions:

  A[i, j] = #{E' subset of E(H_j) : (V(H_j), E') is isomorphic to H_i with
             the chosen vertex x of orbit j in orbit i}

and inverts it exactly over the integers (A is unit upper-triangular in the
paper's orbit order, so back-substitution needs no division).

The patterns and the printed orbit labels are transcribed from the figure
of all vertex orbits (Fig. node_orbits); orbits of unlabelled vertices follow
from automorphisms (Definition "auto").

Run ``python -m paper_1911_10616_amd.gen_tables`` to rewrite the header.
"""
from __future__ import annotations

import itertools
import os

# H0..H29: (edges on 1-based node ids, {node: printed orbit label})
_PATTERNS = (
    ((12,), {2: 0}),
    ((12, 23), {2: 2, 3: 1}),
    ((12, 13, 23), {3: 3}),
    ((12, 23, 34), {3: 5, 4: 4}),
    ((13, 23, 34), {3: 7, 4: 6}),
    ((12, 13, 24, 34), {3: 8}),
    ((12, 23, 24, 34), {1: 9, 2: 11, 3: 10}),
    ((12, 13, 14, 24, 34), {2: 12, 4: 13}),
    ((12, 13, 14, 23, 24, 34), {4: 14}),
    ((12, 23, 34, 45), {3: 17, 4: 16, 5: 15}),
    ((13, 23, 34, 45), {1: 19, 3: 21, 4: 20, 5: 18}),
    ((13, 23, 34, 35), {3: 23, 5: 22}),
    ((13, 24, 34, 35, 45), {1: 24, 3: 26, 5: 25}),
    ((12, 13, 23, 34, 45), {1: 29, 3: 30, 4: 28, 5: 27}),
    ((13, 23, 34, 35, 45), {1: 31, 3: 33, 4: 32}),
    ((12, 13, 24, 35, 45), {5: 34}),
    ((12, 23, 24, 35, 45), {1: 35, 2: 38, 3: 37, 5: 36}),
    ((12, 23, 24, 25, 35, 45), {1: 39, 2: 42, 3: 40, 5: 41}),
    ((12, 13, 23, 34, 35, 45), {3: 44, 4: 43}),
    ((12, 23, 24, 34, 35, 45), {1: 45, 2: 47, 3: 48, 5: 46}),
    ((12, 13, 14, 25, 35, 45), {1: 50, 2: 49}),
    ((12, 13, 24, 34, 35, 45), {1: 51, 3: 53, 5: 52}),
    ((13, 14, 23, 24, 34, 35, 45), {1: 54, 3: 55}),
    ((12, 23, 24, 25, 34, 35, 45), {1: 56, 2: 58, 3: 57}),
    ((12, 13, 23, 24, 34, 35, 45), {1: 59, 2: 60, 3: 61}),
    ((12, 13, 14, 25, 34, 35, 45), {2: 62, 3: 64, 5: 63}),
    ((12, 13, 23, 24, 25, 34, 35, 45), {1: 65, 3: 67, 5: 66}),
    ((12, 13, 14, 23, 25, 34, 35, 45), {3: 69, 4: 68}),
    ((12, 13, 14, 23, 24, 25, 34, 35, 45), {1: 70, 4: 71}),
    ((12, 13, 14, 15, 23, 24, 25, 34, 35, 45), {5: 72}),
)
NORB = 73


def _edges(code):
    return [(c // 10 - 1, c % 10 - 1) for code_ in [code] for c in code_]


def _canon(k, edges):
    return frozenset(frozenset(e) for e in edges)


def patterns():
    """[(k, edge set, orbit per node)] derived by automorphisms."""
    out = []
    for code, lab in _PATTERNS:
        edges = _edges(code)
        k = 1 + max(max(e) for e in edges)
        es = _canon(k, edges)
        autos = [p for p in itertools.permutations(range(k))
                 if _canon(k, [(p[a], p[b]) for a, b in edges]) == es]
        orbit = []
        for x in range(k):
            labels = {lab[y + 1] for y in {p[x] for p in autos} if y + 1 in lab}
            if len(labels) != 1:
                raise ValueError("figure transcription inconsistent")
            orbit.append(labels.pop())
        out.append((k, es, orbit))
    return out


def transform():
    """A as a dict {(i, j): value} (integers)."""
    pats = patterns()
    by_k = {}
    for h, (k, es, orbit) in enumerate(pats):
        by_k.setdefault(k, []).append(h)
    A = {}
    for j_h, (k, es, orbit_j) in enumerate(pats):
        elist = sorted(tuple(sorted(e)) for e in es)
        for x in range(k):
            oj = orbit_j[x]
            if any(key[1] == oj for key in A):
                continue  # one representative vertex per orbit
            for r in range(len(elist) + 1):
                for sub in itertools.combinations(elist, r):
                    sub_es = _canon(k, sub)
                    for i_h in by_k[k]:
                        kk, es_i, orbit_i = pats[i_h]
                        if len(es_i) != len(sub_es):
                            continue
                        hit = None
                        for p in itertools.permutations(range(k)):  # node of H_i -> vertex
                            if _canon(k, [(p[a], p[b]) for a, b in (tuple(e) for e in es_i)]) == sub_es:
                                hit = p
                                break
                        if hit is None:
                            continue
                        oi = orbit_i[hit.index(x)]
                        A[(oi, oj)] = A.get((oi, oj), 0) + 1
                        break
    return A


def inverse(A):
    """Exact inverse of the unit upper-triangular A (dict form)."""
    n = NORB
    M = [[A.get((i, j), 0) for j in range(n)] for i in range(n)]
    for i in range(n):
        if M[i][i] != 1 or any(M[i][j] for j in range(i)):
            raise ValueError("A is not unit upper-triangular")
    inv = [[0] * n for _ in range(n)]
    for c in range(n):  # solve M y = e_c by back-substitution
        y = [0] * n
        for i in range(n - 1, -1, -1):
            y[i] = (1 if i == c else 0) - sum(M[i][j] * y[j] for j in range(i + 1, n))
        for i in range(n):
            inv[i][c] = y[i]
    return inv


def orbit_tables():
    """(pattern of each orbit, number of pattern vertices in each orbit)."""
    pat = [0] * NORB
    size = [0] * NORB
    for h, (k, es, orbit) in enumerate(patterns()):
        for o in orbit:
            pat[o] = h
            size[o] += 1
    return pat, size


def header_text():
    A = transform()
    inv = inverse(A)
    opat, osize = orbit_tables()
    rows = []
    ptr = [0]
    for i in range(NORB):
        for j in range(NORB):
            if inv[i][j]:
                rows.append((j, inv[i][j]))
        ptr.append(len(rows))
    lines = [
        "/* Generated by paper_1911_10616_amd/gen_tables.py -- do not edit. */",
        "/* Inverse of the induced->non-induced orbit transform A (paper appendix",
        " * 'Conversion between Induced and Noninduced counts'): induced = Ainv *",
        " * non-induced, row by row, in uint64 wrap-around arithmetic.  Sparse",
        " * rows: entries ORB_AINV_PTR[i] .. ORB_AINV_PTR[i+1]-1. */",
        "#pragma once",
        "#include <stdint.h>",
        f"#define ORB_AINV_NNZ {len(rows)}",
        "static const uint16_t ORB_AINV_PTR[74] = {" + ", ".join(map(str, ptr)) + "};",
        "static const uint8_t ORB_AINV_COL[ORB_AINV_NNZ] = {" + ", ".join(str(c) for c, _ in rows) + "};",
        "static const int16_t ORB_AINV_VAL[ORB_AINV_NNZ] = {" + ", ".join(str(v) for _, v in rows) + "};",
        "/* Pattern H_h of each orbit and the number of its vertices in the orbit",
        " * (Fig. node_orbits, orbits of unlabelled vertices by automorphisms). */",
        "#define ORB_NPATTERN 30",
        "static const uint8_t ORB_ORBIT_PATTERN[73] = {" + ", ".join(map(str, opat)) + "};",
        "static const uint8_t ORB_ORBIT_SIZE[73] = {" + ", ".join(map(str, osize)) + "};",
        "",
    ]
    return "\n".join(lines)


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "orbit_tables.h")
    with open(path, "w") as f:
        f.write(header_text())
    print("wrote", path)


if __name__ == "__main__":
    main()
