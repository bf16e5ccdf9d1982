"""Asynchronous counts (ORB_ASYNC): orbit_prepare fixes the sizes once, then
orbit_count_ex enqueues the whole count with no host synchronisation and
orbit_count_status reports the outcome.  Bit-exact against the oracle and
the synchronous path."""
import time

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


@pytest.mark.parametrize("name,make", [("er", lambda: gg.erdos_renyi(40, 0.3, 9101)),
                                       ("ba", lambda: gg.barabasi_albert(300, 4, 9102)),
                                       ("chunglu", lambda: gg.chung_lu(800, 8.0, 2.1, 100.0, 3200, 9103)),
                                       ("K12", lambda: gg.complete(12))])
def test_async_counts_match_oracle(orbit, name, make):
    import torch
    rp, ci = make()
    print("async", name, flush=True)
    s = torch.cuda.Stream()
    c = orbit.Counter(rp, ci, 5, stream=s, asynchronous=True)
    c.run()
    c.status()
    got = c.out[: c.n].cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, oracle.induced_counts(rp, ci, threads=8))


def test_async_returns_before_the_work_ends(orbit):
    """On a graph whose count takes a fraction of a second the call returns
    while the stream is still busy; the status call then waits, and the
    counts equal the synchronous path's."""
    import torch
    rp, ci = gg.chung_lu(200_000, 20.0, 2.1, 5000.0, 2_000_000, 9104)
    ref = orbit.Counter(rp, ci, 5).run().clone()
    s = torch.cuda.Stream()
    c = orbit.Counter(rp, ci, 5, stream=s, asynchronous=True)
    c.run()
    c.status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.run()
    t_call = time.perf_counter() - t0
    busy = not s.query()
    t1 = time.perf_counter()
    c.status()
    t_wait = time.perf_counter() - t1
    print(f"call {t_call * 1e3:.2f} ms, busy after return {busy}, wait {t_wait * 1e3:.1f} ms",
          flush=True)
    assert busy and t_wait > t_call
    assert torch.equal(c.out[: c.n], ref)


def test_async_sizes_of_another_graph_are_reported(orbit):
    """Sizes prepared for one graph, counted on another of the same n and m
    with more triangles: the count reports ORB_E_INTERNAL."""
    import ctypes
    import torch
    n = 120
    rp1, ci1 = gg.from_edge_list(n, [(3 * t + i, 3 * t + j) for t in range(40)
                                     for i, j in ((0, 1), (0, 2), (1, 2))])
    rp2, ci2 = gg.complete(16)
    rp2 = np.concatenate([rp2, np.full(n - 16, rp2[-1], np.uint32)])
    c = orbit.Counter(rp1, ci1, 5, asynchronous=True)
    c.rp.copy_(torch.as_tensor(rp2.view(np.int32)))
    c.ci.copy_(torch.as_tensor(ci2.view(np.int32)))
    c.run()
    with pytest.raises(orbit.OrbError) as e:
        c.status()
    assert e.value.status == -9
    c.rp.copy_(torch.as_tensor(rp1.view(np.int32)))
    c.ci.copy_(torch.as_tensor(ci1.view(np.int32)))
    c.run()
    c.status()
    np.testing.assert_array_equal(c.out[:n].cpu().numpy().view(np.uint64),
                                  oracle.induced_counts(rp1, ci1))
