"""The Chung-Lu 1M workload at full size, in the launch configuration that
bench.py times (learned schedule, default workgroup count), checked through
properties that hold at any size -- the oracle cannot enumerate the
5-vertex neighbourhoods of this graph one vertex at a time, since nearly
every vertex is within two hops of a hub with tens of thousands of
neighbours.

* orbit 0 is the degree; orbits 1-3 satisfy the degree identities
  I2 + I3 = C(d,2) and I1 + 2 I3 = sum_{v~u} (d(v) - 1);
* the non-induced counts A I (A: the oracle's transform) of the star
  orbits are the closed forms C(d,3), C(d,4), sum_{v~u} C(d(v)-1, 2) and
  sum_{v~u} C(d(v)-1, 3);
* summed over vertices, the orbits of one pattern give the same number of
  copies (sum_u I_o(u) / |o| equal across the orbits of a pattern);
* relabelling the vertices permutes the rows: the run on the same graph
  with ids permuted at random (a different order of every kernel's work)
  gives exactly the permuted counts, all 73 orbits of all 10^6 vertices.

All comparisons are exact in uint64 (modulo 2^64).
"""
import numpy as np
import pytest

import oracle
from paper_1911_10616_amd import graphgen as gg

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

U = np.uint64


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_10616_amd import orbit
    import bench
    w, _ = bench.train_cost_model(orbit)
    rp, ci = gg.workload("chunglu1m")
    print("chunglu1m generated", len(rp) - 1, ci.size // 2, flush=True)
    c = orbit.Counter(rp, ci, 5, schedule="mlp", mlp_weights=w)
    counts = c.run().cpu().numpy().view(U).copy()
    del c
    torch.cuda.empty_cache()
    print("chunglu1m counted", flush=True)
    return orbit, w, rp, ci, counts


def _binom(x, k):
    x = x.astype(U)
    out = np.ones_like(x)
    for i in range(k):
        out = out * np.where(x >= U(i), x - U(i), U(0))
    den = U([1, 1, 2, 6, 24][k])
    return out // den  # the product of k consecutive integers < 2^64 here


def _row_sums(rp, vals):
    cs = np.zeros(vals.size + 1, dtype=U)
    np.cumsum(vals.astype(U), out=cs[1:])
    return cs[rp[1:].astype(np.int64)] - cs[rp[:-1].astype(np.int64)]


def test_degree_identities(setup):
    _, _, rp, ci, I = setup
    d = np.diff(rp).astype(U)
    np.testing.assert_array_equal(I[:, 0], d)
    assert np.array_equal(I[:, 2] + I[:, 3], _binom(d, 2))
    nb = d[ci.astype(np.int64)]
    assert np.array_equal(I[:, 1] + U(2) * I[:, 3], _row_sums(rp, nb - U(1)))


def test_star_orbits_closed_forms(setup):
    _, _, rp, ci, I = setup
    A = oracle.transform_matrix().astype(U)
    d = np.diff(rp).astype(U)
    nb = d[ci.astype(np.int64)]
    def noninduced(o):
        return (I * A[o][None, :]).sum(axis=1, dtype=U)
    assert np.array_equal(noninduced(7), _binom(d, 3))   # 3-star centre
    assert np.array_equal(noninduced(23), _binom(d, 4))  # 4-star centre
    assert np.array_equal(noninduced(6), _row_sums(rp, _binom(nb - U(1), 2)))   # 3-star leaf
    assert np.array_equal(noninduced(22), _row_sums(rp, _binom(nb - U(1), 3)))  # 4-star leaf


def test_pattern_copies_agree_across_orbits(setup):
    _, _, _, _, I = setup
    t = oracle.tables()
    g = np.asarray(t["orbit_graphlet"])
    size = np.asarray(t["orbit_size"]).astype(U)
    tot = I.sum(axis=0, dtype=U)
    for pat in np.unique(g):
        orbs = np.flatnonzero(g == pat)
        for o1, o2 in zip(orbs[:-1], orbs[1:]):
            assert tot[o1] * size[o2] == tot[o2] * size[o1], (pat, o1, o2)


def test_relabelled_graph_gives_permuted_counts(setup):
    import torch
    orbit, w, rp, ci, I = setup
    seed = gg.CONFIG_SEED_BASE + 6
    rp2, ci2 = gg.workload("chunglu1m_perm")
    perm = np.random.Generator(np.random.PCG64(seed)).permutation(len(rp) - 1)
    c = orbit.Counter(rp2, ci2, 5, schedule="mlp", mlp_weights=w)
    I2 = c.run().cpu().numpy().view(U)
    del c
    torch.cuda.empty_cache()
    bad = np.flatnonzero((I2[perm] != I).any(axis=1))
    assert bad.size == 0, f"{bad.size} vertices differ, first {bad[:5]}"
    # the library's own renumbering (heaviest degree class first) on the
    # permuted graph: the same counts under the caller's ids
    c = orbit.Counter(rp2, ci2, 5, schedule="mlp", mlp_weights=w, relabel=True)
    I3 = c.run().cpu().numpy().view(U)
    del c
    torch.cuda.empty_cache()
    bad = np.flatnonzero((I3 != I2).any(axis=1))
    assert bad.size == 0, f"relabelled: {bad.size} vertices differ, first {bad[:5]}"
