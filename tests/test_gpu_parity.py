"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer work: every comparison is bit-exact (uint64, modulo 2^64).
"""
import numpy as np
import pytest

import oracle
from paper_1911_10616_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orbit():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_10616_amd import orbit as o
    return o


def _say(*a):
    print(*a, flush=True)


def _cases():
    out = []
    for s in range(24):
        n = 8 + (s * 7) % 33
        p = [0.15, 0.3, 0.5, 0.7][s % 4]
        out.append((f"er_n{n}_p{p}_s{s}", lambda n=n, p=p, s=s: gg.erdos_renyi(n, p, 9000 + s)))
    for s in range(4):
        out.append((f"ba_{s}", lambda s=s: gg.barabasi_albert(60 + 20 * s, 3, 100 + s)))
    out.append(("chunglu_small", lambda: gg.chung_lu(400, 8.0, 2.1, 60.0, 1600, 3)))
    out.append(("rmat_9", lambda: gg.rmat(9, 8, seed=4)))
    return out


@pytest.mark.parametrize("name,make", _cases(), ids=[c[0] for c in _cases()])
def test_random_graphs_induced(orbit, name, make):
    rp, ci = make()
    _say("case", name, len(rp) - 1, ci.size // 2)
    ref = oracle.induced_counts(rp, ci, threads=8)
    got = orbit.count_np(rp, ci, 5)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("seed", range(8))
def test_random_graphs_noninduced(orbit, seed):
    rp, ci = gg.erdos_renyi(10 + seed, [0.3, 0.5, 0.7, 0.9][seed % 4], 7000 + seed)
    _say("noninduced seed", seed)
    np.testing.assert_array_equal(orbit.count_np(rp, ci, 5, noninduced=True),
                                  oracle.noninduced_counts(rp, ci))


@pytest.mark.parametrize("k_max", [3, 4])
def test_smaller_kmax(orbit, k_max):
    K = orbit.num_orbits(k_max)
    for s in range(4):
        rp, ci = gg.erdos_renyi(30, 0.25, 8000 + s)
        _say("kmax", k_max, "seed", s)
        ref = oracle.induced_counts(rp, ci, kmax=k_max)[:, :K]
        np.testing.assert_array_equal(orbit.count_np(rp, ci, k_max), ref)
        refn = oracle.noninduced_counts(rp, ci, kmax=k_max)[:, :K]
        np.testing.assert_array_equal(orbit.count_np(rp, ci, k_max, noninduced=True), refn)


def _special():
    return [
        ("single_vertex", lambda: gg.csr_from_edges(1, [], [])),
        ("empty5", lambda: gg.csr_from_edges(5, [], [])),
        ("one_edge", lambda: gg.from_edge_list(2, [(0, 1)])),
        ("isolated_mix", lambda: gg.from_edge_list(9, [(0, 3), (3, 5), (5, 0), (7, 8)])),
        ("K8", lambda: gg.complete(8)),
        ("K12", lambda: gg.complete(12)),
        ("C5", lambda: gg.cycle(5)),
        ("C9", lambda: gg.cycle(9)),
        ("star40", lambda: gg.star(40)),
        ("K_5_7", lambda: gg.complete_bipartite(5, 7)),
        ("path10", lambda: gg.path(10)),
    ]


@pytest.mark.parametrize("name,make", _special(), ids=[c[0] for c in _special()])
def test_special_graphs(orbit, name, make):
    rp, ci = make()
    _say("special", name)
    np.testing.assert_array_equal(orbit.count_np(rp, ci, 5), oracle.induced_counts(rp, ci))


def test_hub_larger_than_lds_tile(orbit):
    # K420: out-degrees up to 419, clique bit rows of 7 words per row (the
    # global-memory rows of larger out-degrees run in the small-tile build)
    rp, ci = gg.complete(420)
    _say("K420")
    got = orbit.count_np(rp, ci, 5)
    from math import comb
    assert (got[:, 0] == 419).all() and (got[:, 3] == comb(419, 2)).all()
    assert (got[:, 14] == comb(419, 3)).all() and (got[:, 72] == comb(419, 4)).all()
    assert (np.delete(got, [0, 3, 14, 72], axis=1) == 0).all()


def _book(k):
    """k triangles sharing the edge (0, 1): spine 0, 1; pages 2 .. k+1."""
    pages = np.arange(2, k + 2)
    u = np.concatenate([[0], np.zeros(k, np.int64), np.ones(k, np.int64)])
    v = np.concatenate([[1], pages, pages])
    return gg.csr_from_edges(k + 2, u, v)


def _book_counts(k):
    """Induced counts of the book with k pages, from the oracle on books with
    4..8 pages: every count of a spine vertex or a page is a sum of
    C(k, j) c_j (j <= 4) over the pages a 2..5-vertex subset takes, hence a
    polynomial of degree <= 4 in k, fixed exactly by five values."""
    from fractions import Fraction
    ks = [4, 5, 6, 7, 8]
    spine = [oracle.induced_counts(*_book(j))[0].astype(object) for j in ks]
    page = [oracle.induced_counts(*_book(j))[2].astype(object) for j in ks]
    def interp(rows):
        out = []
        for o in range(73):
            tot = Fraction(0)
            for i, xi in enumerate(ks):
                term = Fraction(int(rows[i][o]))
                for j, xj in enumerate(ks):
                    if j != i:
                        term *= Fraction(k - xj, xi - xj)
                tot += term
            assert tot.denominator == 1
            out.append(int(tot) % (1 << 64))
        return np.array(out, dtype=np.uint64)
    exp = np.empty((k + 2, 73), dtype=np.uint64)
    exp[0] = exp[1] = interp(spine)
    exp[2:] = interp(page)
    return exp


@pytest.mark.parametrize("k", [70, 300, 5000])
def test_book_long_triangle_lists(orbit, k):
    """One edge in k triangles: its triangle list is sorted in registers
    (<= 64), in LDS (<= 4096) or by the bitmap counting sort (> 4096)."""
    _say("book", k)
    rp, ci = _book(k)
    exp = _book_counts(k)
    np.testing.assert_array_equal(orbit.count_np(rp, ci, 5), exp)
    rp2, ci2 = gg.relabel(rp, ci, 77)
    perm = np.random.Generator(np.random.PCG64(77)).permutation(k + 2)
    np.testing.assert_array_equal(orbit.count_np(rp2, ci2, 5)[perm], exp)


def test_er2000_full(orbit):
    """The ER(n=2000, p=0.005) workload, every vertex and orbit."""
    rp, ci = gg.workload("er2000")
    _say("er2000")
    ref = oracle.induced_counts(rp, ci, threads=16)
    np.testing.assert_array_equal(orbit.count_np(rp, ci, 5), ref)


def test_entry_points_agree_and_deterministic(orbit):
    rp, ci = gg.barabasi_albert(300, 4, 11)
    _say("entry points")
    a = orbit.count_minimal(rp, ci, 5)
    c = orbit.Counter(rp, ci, 5)
    b1 = c.run().cpu().numpy().view(np.uint64).copy()
    b2 = c.run().cpu().numpy().view(np.uint64).copy()
    np.testing.assert_array_equal(a, b1)
    np.testing.assert_array_equal(b1, b2)
    # a different number of persistent workgroups changes only the schedule
    b3 = orbit.count_np(rp, ci, 5, num_wg=7)
    np.testing.assert_array_equal(b1, b3)


def _bad_inputs():
    good_rp, good_ci = gg.from_edge_list(4, [(0, 1), (1, 2), (2, 3), (0, 2)])
    rp = good_rp.copy(); ci = good_ci.copy()
    cases = []
    c = ci.copy(); c[0], c[1] = c[1], c[0]
    cases.append(("unsorted", rp, c, -2))
    c = ci.copy(); c[0] = 0  # vertex 0 lists itself
    cases.append(("self_loop", rp, c, -3))
    c = ci.copy(); c[1] = c[0]
    cases.append(("duplicate", rp, c, -4))
    # asymmetric: 0-3 only in 0's list
    r2, c2 = gg.path(4)
    c2 = c2.copy(); c2[0] = 3  # vertex 0 now lists 3, which does not list 0
    cases.append(("asymmetric", r2, c2, -5))
    c = ci.copy(); c[-1] = 17
    cases.append(("out_of_range", rp, c, -6))
    r = rp.copy(); r[2] = r[3] + 1
    cases.append(("rowptr", r, ci, -6))
    return cases


@pytest.mark.parametrize("name,rp,ci,code", _bad_inputs(), ids=[c[0] for c in _bad_inputs()])
def test_malformed_input_rejected(orbit, name, rp, ci, code):
    import torch
    _say("bad input", name)
    drp, dci = orbit._dev_csr(rp, ci)
    n = len(rp) - 1
    m = int(rp[-1]) // 2
    out = torch.zeros((n, 73), dtype=torch.int64, device="cuda")
    ws = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    st, _ = orbit.raw_count_ex(drp.data_ptr(), dci.data_ptr(), n, m, 5, out.data_ptr(),
                               ws.data_ptr(), ws.numel())
    assert st == code


def test_argument_errors(orbit):
    import torch
    rp, ci = gg.cycle(6)
    drp, dci = orbit._dev_csr(rp, ci)
    out = torch.zeros((6, 73), dtype=torch.int64, device="cuda")
    ws = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    st, _ = orbit.raw_count_ex(drp.data_ptr(), dci.data_ptr(), 6, 6, 6, out.data_ptr(),
                               ws.data_ptr(), ws.numel())
    assert st == -1  # k_max
    st, need = orbit.raw_count_ex(drp.data_ptr(), dci.data_ptr(), 6, 6, 5, out.data_ptr(),
                                  ws.data_ptr(), 1024)
    assert st == -7 and need > 1024  # workspace
    st, _ = orbit.raw_count_ex(drp.data_ptr(), dci.data_ptr(), 6, 6, 5, out.data_ptr(),
                               ws.data_ptr(), ws.numel(), flags=0x80)
    assert st == -1  # unknown flag


@pytest.mark.parametrize("groups", ["wg", "wave"])
def test_execution_groups(orbit, groups):
    """A workgroup per source and a wave per source give the same counts."""
    graphs = [gg.erdos_renyi(40, 0.3, 11), gg.barabasi_albert(150, 3, 12),
              gg.chung_lu(500, 8.0, 2.1, 80.0, 2000, 13), gg.complete(12), _book(70)]
    for i, (rp, ci) in enumerate(graphs):
        _say("groups", groups, "graph", i)
        np.testing.assert_array_equal(orbit.count_np(rp, ci, 5, groups=groups),
                                      oracle.induced_counts(rp, ci, threads=8))
        np.testing.assert_array_equal(orbit.count_np(rp, ci, 5, noninduced=True, groups=groups),
                                      oracle.noninduced_counts(rp, ci, threads=8))


def test_relabelled_counting(orbit):
    """ORB_RELABEL: counting on the renumbered copy gives the caller's counts
    (rows of up to 64 sorted in registers, up to 4096 in LDS, longer ones by
    bitmap: the books of 300 and 5000 pages have such rows)."""
    graphs = [gg.relabel(*gg.chung_lu(800, 8.0, 2.1, 120.0, 3200, 71), 9),
              gg.barabasi_albert(200, 3, 72), gg.erdos_renyi(40, 0.4, 73), gg.complete(12)]
    for i, (rp, ci) in enumerate(graphs):
        _say("relabel graph", i)
        np.testing.assert_array_equal(orbit.count_np(rp, ci, 5, relabel=True),
                                      oracle.induced_counts(rp, ci, threads=8))
        np.testing.assert_array_equal(orbit.count_np(rp, ci, 5, noninduced=True, relabel=True),
                                      oracle.noninduced_counts(rp, ci, threads=8))
    for k in (300, 5000):
        _say("relabel book", k)
        rp, ci = gg.relabel(*_book(k), 5)
        perm = np.random.Generator(np.random.PCG64(5)).permutation(k + 2)
        got = orbit.count_np(rp, ci, 5, relabel=True)
        np.testing.assert_array_equal(got[perm], _book_counts(k))
    rp, ci = gg.erdos_renyi(30, 0.3, 74)
    np.testing.assert_array_equal(orbit.count_np(rp, ci, 4, relabel=True),
                                  oracle.induced_counts(rp, ci, kmax=4)[:, :15])


def test_relabel_argument_errors(orbit):
    import torch
    rp, ci = gg.complete(6)
    feat = torch.empty((6, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(orbit.OrbError):
        orbit.Counter(rp, ci, 5, relabel=True, features_out=feat).run()
    vptr, brp, bci = gg.batch_small(4, 3, nmin=5, nmax=8)
    with pytest.raises(orbit.OrbError):
        c = orbit.BatchCounter(vptr, brp, bci, 5)
        c.opts.flags |= orbit.ORB_RELABEL
        c.run()


@pytest.mark.parametrize("groups", ["wg", "wave"])
def test_orbit_groups_serial_and_overlapped(orbit, groups):
    """The three 5-vertex orbit groups overlapped (the default: two of them
    on a helper stream beside the pair sweep) or run one after another give
    the oracle's counts."""
    graphs = [gg.erdos_renyi(40, 0.3, 8101), gg.barabasi_albert(200, 3, 8102),
              gg.chung_lu(500, 8.0, 2.1, 80.0, 2000, 8103), gg.complete(12)]
    for i, (rp, ci) in enumerate(graphs):
        _say("orbit groups", groups, i)
        ref = oracle.induced_counts(rp, ci, threads=8)
        np.testing.assert_array_equal(orbit.count_np(rp, ci, 5, groups=groups, serial=True), ref)
        np.testing.assert_array_equal(orbit.count_np(rp, ci, 5, groups=groups), ref)
