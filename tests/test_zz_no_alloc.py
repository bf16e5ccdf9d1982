"""orbit_count_noalloc: the entry point for callers that cannot allocate.

Its workspace is the library's static device buffer, so it is checked
against orbit_count_ex (caller's workspace, same kernels) and the oracle,
bit for bit, on two calls in a row -- the second on a smaller graph, with
the buffer still holding the first call's contents -- and on inputs it
must reject.
"""
import ctypes

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


def _raw_noalloc(orbit, rp, ci, k_max=5):
    """One call through the C ABI; returns (status, counts as uint64)."""
    import torch
    drp, dci = orbit._dev_csr(rp, ci)
    n = len(rp) - 1
    m = int(rp[-1]) // 2
    out = torch.full((max(n, 1), orbit.num_orbits(k_max)), -1, dtype=torch.int64,
                     device="cuda")
    st = orbit._lib.orbit_count_noalloc(ctypes.c_void_p(drp.data_ptr()),
                                        ctypes.c_void_p(dci.data_ptr()), n, m, k_max,
                                        ctypes.c_void_p(out.data_ptr()), None)
    torch.cuda.synchronize()
    return st, out[:n].cpu().numpy().view(np.uint64)


def test_noalloc_matches_count_ex_twice(orbit):
    assert orbit._lib.orbit_noalloc_capacity() == 64 << 20
    graphs = [gg.erdos_renyi(400, 0.04, 5101), gg.barabasi_albert(150, 3, 5102)]
    for i, (rp, ci) in enumerate(graphs):
        print("noalloc call", i, len(rp) - 1, ci.size // 2, flush=True)
        st, got = _raw_noalloc(orbit, rp, ci)
        assert st == 0
        ref = orbit.to_u64(orbit.Counter(rp, ci, 5).run())
        np.testing.assert_array_equal(got, ref)
        np.testing.assert_array_equal(got, oracle.induced_counts(rp, ci, threads=8))
    st, got = _raw_noalloc(orbit, *graphs[1], k_max=4)
    assert st == 0
    np.testing.assert_array_equal(got, oracle.induced_counts(*graphs[1], kmax=4)[:, :15])


def test_noalloc_rejects_what_does_not_fit(orbit):
    import torch
    # n alone is too large: rejected before any kernel runs
    n = 20_000_000
    rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    st = orbit._lib.orbit_count_noalloc(ctypes.c_void_p(rp.data_ptr()),
                                        ctypes.c_void_p(ci.data_ptr()), n, 0, 5,
                                        ctypes.c_void_p(out.data_ptr()), None)
    assert st == -11
    del rp
    # phase 1 fits, the counts (584 bytes per vertex) do not
    rp2, ci2 = gg.cycle(300_000)
    st, _ = _raw_noalloc(orbit, rp2, ci2)
    assert st == -11
    assert "static buffer" in orbit._lib.orbit_strerror(-11).decode()
    # a malformed graph is still rejected as such
    rp3, ci3 = gg.path(6)
    ci3 = ci3.copy()
    ci3[1], ci3[2] = ci3[2], ci3[1]  # vertex 1 lists (2, 0)
    st, _ = _raw_noalloc(orbit, rp3, ci3)
    assert st == -2
    # and the buffer still counts correctly afterwards
    rp4, ci4 = gg.erdos_renyi(60, 0.2, 5103)
    st, got = _raw_noalloc(orbit, rp4, ci4)
    assert st == 0
    np.testing.assert_array_equal(got, oracle.induced_counts(rp4, ci4))
