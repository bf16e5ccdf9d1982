"""Edge orbit counts E0..E11 per CSR slot (orbit_count_edges) against the
oracle's enumeration, bit-exact, through the C ABI."""
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


def _book(k):
    pages = np.arange(2, k + 2)
    u = np.concatenate([[0], np.zeros(k, np.int64), np.ones(k, np.int64)])
    v = np.concatenate([[1], pages, pages])
    return gg.csr_from_edges(k + 2, u, v)


def _graphs():
    out = [(f"er_{s}", lambda s=s: gg.erdos_renyi(12 + 5 * s, [0.2, 0.4, 0.6][s % 3], 7700 + s))
           for s in range(6)]
    out += [("ba200", lambda: gg.barabasi_albert(200, 3, 7710)),
            ("chunglu_small", lambda: gg.chung_lu(400, 8.0, 2.1, 60.0, 1600, 7711)),
            ("rmat_9", lambda: gg.rmat(9, 8, seed=7712)),
            ("K9", lambda: gg.complete(9)), ("C7", lambda: gg.cycle(7)),
            ("star12", lambda: gg.star(12)), ("K_4_6", lambda: gg.complete_bipartite(4, 6)),
            ("book70", lambda: _book(70)),
            ("isolated_mix", lambda: gg.from_edge_list(9, [(0, 3), (3, 5), (5, 0), (7, 8)]))]
    return out


@pytest.mark.parametrize("k_max", [4, 5])
@pytest.mark.parametrize("name,make", _graphs(), ids=[g[0] for g in _graphs()])
def test_edge_orbits_match_oracle(orbit, name, make, k_max):
    rp, ci = make()
    print("edges", name, k_max, flush=True)
    vc, ec = orbit.count_edges(rp, ci, k_max)
    np.testing.assert_array_equal(orbit.to_u64(ec), oracle.edge_counts(rp, ci, threads=8))
    K = orbit.num_orbits(k_max)
    np.testing.assert_array_equal(orbit.to_u64(vc),
                                  oracle.induced_counts(rp, ci, kmax=k_max, threads=8)[:, :K])


@pytest.mark.parametrize("name,make", [("er60_dense", lambda: gg.erdos_renyi(60, 0.7, 7720)),
                                       ("book200", lambda: _book(200))])
def test_edge_orbits_small_tiles(orbit, name, make):
    """The small-tile build: global clique rows and 4-cycle paths of hubs."""
    rp, ci = make()
    print("edges tiles", name, flush=True)
    with orbit.using_library():
        _, ec = orbit.count_edges(rp, ci, 4)
    np.testing.assert_array_equal(orbit.to_u64(ec), oracle.edge_counts(rp, ci, threads=8))


def test_edge_orbit_arguments(orbit):
    import ctypes
    import torch
    rp, ci = gg.complete(6)
    c = orbit.Counter(rp, ci, 4)
    e = torch.empty((30, 12), dtype=torch.int64, device="cuda")
    need = ctypes.c_uint64(0)

    def call(k_max, edges, opts):
        return orbit._lib.orbit_count_edges(
            ctypes.c_void_p(c.rp.data_ptr()), ctypes.c_void_p(c.ci.data_ptr()), 6, 15, k_max,
            ctypes.c_void_p(c.out.data_ptr()), edges, ctypes.c_void_p(c.ws.data_ptr()),
            c.ws_bytes, ctypes.byref(need), None, ctypes.byref(opts))
    assert call(3, ctypes.c_void_p(e.data_ptr()), c.opts) == -1
    assert call(4, None, c.opts) == -1
    o = orbit._opts(relabel=True)
    assert call(4, ctypes.c_void_p(e.data_ptr()), o) == -1
    assert call(4, ctypes.c_void_p(e.data_ptr()), c.opts) == 0
