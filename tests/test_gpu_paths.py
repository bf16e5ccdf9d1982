"""GPU regression tests of the paths that only large graphs reach.

* The small-tile build (every LDS tile shrunk) on oracle-sized graphs:
  global clique bit rows, wheel maps in LDS windows and in global memory,
  the LDS and bitmap sorts of long triangle lists.
* The library build on graphs with those features at full size: vertices
  of out-degree 520 (clique rows in global memory, long out-lists in the
  5-cycle kernel), a star whose centre count C(s,4) wraps modulo 2^64, and
  the overflow flags.
* Replaying a plan on a changed input reports an error and writes nothing
  out of bounds.

Every comparison is bit-exact (uint64 modulo 2^64).
"""
from fractions import Fraction
from math import comb

import numpy as np
import pytest

import oracle
from paper_1911_10616_amd import graphgen as gg

pytestmark = pytest.mark.gpu
M64 = 1 << 64


@pytest.fixture(scope="module")
def orbit():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_10616_amd import orbit as o
    return o


def _say(*a):
    print(*a, flush=True)


def _book(k):
    pages = np.arange(2, k + 2)
    u = np.concatenate([[0], np.zeros(k, np.int64), np.ones(k, np.int64)])
    v = np.concatenate([[1], pages, pages])
    return gg.csr_from_edges(k + 2, u, v)


def _hub_over(g):
    """A new vertex 0 joined to every vertex of g (shifted to 1..n)."""
    rp, ci = g
    n = len(rp) - 1
    src = np.repeat(np.arange(n), np.diff(rp.astype(np.int64)))
    u = np.concatenate([src + 1, np.zeros(n, np.int64)])
    v = np.concatenate([ci.astype(np.int64) + 1, np.arange(1, n + 1)])
    return gg.csr_from_edges(n + 1, u, v)


def _tile_graphs():
    return [
        ("er60_dense", lambda: gg.erdos_renyi(60, 0.85, 4101)),   # out-degrees > 32, > 16
        ("er45", lambda: gg.erdos_renyi(45, 0.5, 4102)),
        ("ba120", lambda: gg.barabasi_albert(120, 5, 4103)),      # hubs of degree > 32
        ("chunglu300", lambda: gg.chung_lu(300, 8.0, 2.1, 60.0, 1200, 4104)),
        ("hub120", lambda: _hub_over(gg.erdos_renyi(120, 0.05, 4105))),  # LDS windows
        ("K30", lambda: gg.complete(30)),
        ("book100", lambda: _book(100)),                          # LDS list sort (65..128)
        ("book200", lambda: _book(200)),                          # bitmap list sort (> 128)
    ]


@pytest.mark.parametrize("groups", ["wg", "wave"])
@pytest.mark.parametrize("name,make", _tile_graphs(), ids=[g[0] for g in _tile_graphs()])
def test_small_tile_build(orbit, name, make, groups):
    rp, ci = make()
    _say("small tiles", name, groups, len(rp) - 1, ci.size // 2)
    with orbit.using_library():
        got = orbit.count_np(rp, ci, 5, groups=groups)
        gotn = orbit.count_np(rp, ci, 5, noninduced=True, groups=groups)
    np.testing.assert_array_equal(got, oracle.induced_counts(rp, ci, threads=8))
    np.testing.assert_array_equal(gotn, oracle.noninduced_counts(rp, ci, threads=8))


def _bip_matching(a):
    """K_{a,a} (sides 0..a-1 and a..2a-1) plus a perfect matching inside the
    second side.  The first side peels first, so its vertices have
    out-degree a."""
    A = np.arange(a)
    B = np.arange(a, 2 * a)
    u = np.concatenate([np.repeat(A, a), B[0::2]])
    v = np.concatenate([np.tile(B, a), B[1::2]])
    return gg.csr_from_edges(2 * a, u, v)


def _family_counts(a, make, rows, ks):
    """Counts of the rows (vertex classes) of make(a), from the oracle on
    make(k) for k in ks, extended by Lagrange interpolation: every count is
    a sum over the class sizes a 2..5-vertex subset draws from, a polynomial
    of degree <= 4 in a.  The last k of ks checks the degree bound."""
    vals = {k: oracle.induced_counts(*make(k)) for k in ks}

    def interp(xs, ys, x):
        tot = Fraction(0)
        for i, xi in enumerate(xs):
            term = Fraction(int(ys[i]))
            for j, xj in enumerate(xs):
                if j != i:
                    term *= Fraction(x - xj, xi - xj)
            tot += term
        assert tot.denominator == 1
        return int(tot)

    fit, chk = ks[:-1], ks[-1]
    out = []
    for r in rows:
        row = []
        for o in range(73):
            ys = [vals[k][r(k)][o] for k in fit]
            assert interp(fit, ys, chk) == int(vals[chk][r(chk)][o])
            row.append(interp(fit, ys, a) % M64)
        out.append(np.array(row, dtype=np.uint64))
    return out


def test_outdegree_520(orbit):
    """Out-degree 520: clique rows beyond the LDS tile, 5-cycle middle
    vertices with long out-lists, against oracle counts of the family."""
    a = 520
    rp, ci = _bip_matching(a)
    _say("K_{520,520} + matching")
    rowA, rowB = _family_counts(a, _bip_matching, [lambda k: 0, lambda k: k],
                                [4, 6, 8, 10, 12, 14])
    got = orbit.count_np(rp, ci, 5)
    assert (got[:a] == rowA).all()
    assert (got[a:] == rowB).all()
    gotn = orbit.count_np(rp, ci, 5, noninduced=True)
    A = oracle.transform_matrix().astype(object)
    for row, g in ((rowA, gotn[0]), (rowB, gotn[a])):
        exp = [(sum(int(A[i, j]) * int(row[j]) for j in range(73))) % M64 for i in range(73)]
        assert [int(x) for x in g] == exp


def test_star_wraps_modulo_2_64(orbit):
    """Star with s = 150,000 leaves: the centre's orbit-23 count C(s,4)
    exceeds 2^64 and comes back modulo 2^64; the overflow flags mark the
    centre only, as the oracle's bound does."""
    import torch
    s = 150_000
    rp, ci = gg.star(s)
    _say("star", s)
    flags = torch.full((s + 1,), 7, dtype=torch.uint8, device="cuda")
    got = orbit.to_u64(orbit.count(rp, ci, 5, overflow_flags=flags))
    centre = {0: s, 2: comb(s, 2), 7: comb(s, 3), 23: comb(s, 4) % M64}
    leaf = {0: 1, 1: s - 1, 6: comb(s - 1, 2), 22: comb(s - 1, 3)}
    for r, exp in ((got[0], centre), (got[1], leaf), (got[s], leaf)):
        assert {int(i): int(r[i]) for i in np.nonzero(r)[0]} == exp
    assert (got[1:] == got[1]).all()
    np.testing.assert_array_equal(flags.cpu().numpy(), oracle.overflow_flags(rp, ci))
    gotn = orbit.count_np(rp, ci, 5, noninduced=True)
    assert int(gotn[0, 23]) == comb(s, 4) % M64


def test_overflow_flags_match_oracle(orbit):
    """Flags on graphs far below 2^63 (all zero) and on a graph with a few
    hubs whose bound crosses it, against the oracle's fp64 bound."""
    import torch
    graphs = [gg.erdos_renyi(50, 0.2, 4201), gg.barabasi_albert(500, 4, 4202),
              gg.from_edge_list(60010, [(0, i) for i in range(1, 60001)] +
                                [(1, i) for i in range(60001, 60010)])]
    for rp, ci in graphs:
        n = len(rp) - 1
        _say("flags n", n)
        f = torch.full((n,), 9, dtype=torch.uint8, device="cuda")
        orbit.count(rp, ci, 5, overflow_flags=f)
        np.testing.assert_array_equal(f.cpu().numpy(), oracle.overflow_flags(rp, ci))


def test_plan_replay_on_changed_input_reports_error(orbit):
    """A plan built on one graph and replayed after its CSR was overwritten
    in place with another graph of the same n and m but more triangles:
    the replay reports ORB_E_INTERNAL (the guards stop every kernel whose
    sizes changed); restoring the graph gives the eager counts again."""
    import torch
    n = 120
    # 40 disjoint triangles (m = 120, 40 triangles) ...
    rp1, ci1 = gg.from_edge_list(n, [(3 * t + i, 3 * t + j) for t in range(40)
                                     for i, j in ((0, 1), (0, 2), (1, 2))])
    # ... and K16 beside 104 isolated vertices (m = 120, 560 triangles)
    rp2, ci2 = gg.complete(16)
    rp2 = np.concatenate([rp2, np.full(n - 16, rp2[-1], np.uint32)])
    assert rp2.size == n + 1 and rp2[-1] == rp1[-1] == 240
    c = orbit.Counter(rp1, ci1, 5)
    eager = c.run().clone()
    plan = orbit.Plan(c)
    plan.launch()
    plan.status()
    assert torch.equal(c.out[:n], eager)
    c.rp.copy_(torch.as_tensor(rp2.view(np.int32)))
    c.ci.copy_(torch.as_tensor(ci2.view(np.int32)))
    plan.launch()
    with pytest.raises(orbit.OrbError) as e:
        plan.status()
    assert e.value.status == -9
    c.rp.copy_(torch.as_tensor(rp1.view(np.int32)))
    c.ci.copy_(torch.as_tensor(ci1.view(np.int32)))
    plan.launch()
    plan.status()
    assert torch.equal(c.out[:n], eager)
    plan.close()
