"""CPU-side checks of the library boundary and the product's tables."""
import ctypes
import os
import re

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "orbit_hip.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|uint64_t|const char \*)\s*(orbit_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_1911_10616_amd.build import LIB
    assert os.path.exists(LIB), "build() first"
    lib = ctypes.CDLL(LIB)
    names = _declared_functions()
    assert len(names) >= 6
    for nm in names:
        assert hasattr(lib, nm), nm


def test_host_only_calls():
    from paper_1911_10616_amd import orbit
    assert [orbit.num_orbits(k) for k in (2, 3, 4, 5, 6)] == [0, 4, 15, 73, 0]
    assert orbit._lib.orbit_strerror(-7).decode() == "workspace too small"


def test_generated_header_is_current():
    from paper_1911_10616_amd import gen_tables
    path = os.path.join(ROOT, "paper_1911_10616_amd", "csrc", "orbit_tables.h")
    assert open(path).read() == gen_tables.header_text()


def test_product_transform_matches_oracle_definition():
    """The product derives A from the pattern definitions with its own code;
    it must equal the oracle's A, which is pinned to Fig. A."""
    from paper_1911_10616_amd import gen_tables
    A = gen_tables.transform()
    M = np.zeros((73, 73), np.int64)
    for (i, j), v in A.items():
        M[i, j] = v
    np.testing.assert_array_equal(M, oracle.transform_matrix())
    inv = np.array(gen_tables.inverse(A), dtype=np.int64)
    np.testing.assert_array_equal(M @ inv, np.eye(73, dtype=np.int64))


def test_product_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_1911_10616_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "orbit_oracle" not in txt, f


def test_orbit_tables_match_oracle():
    """The product's orbit -> pattern and orbit-size tables (its own
    transcription) agree with the oracle's."""
    from paper_1911_10616_amd import gen_tables
    pat, size = gen_tables.orbit_tables()
    t = oracle.tables()
    assert list(pat) == [int(x) for x in t["orbit_graphlet"]]
    assert list(size) == [int(x) for x in t["orbit_size"]]


def test_every_status_has_a_message():
    from paper_1911_10616_amd import orbit
    msgs = [orbit._lib.orbit_strerror(c).decode() for c in range(0, -12, -1)]
    assert all(m and m != "unknown status" for m in msgs), msgs
    assert len(set(msgs)) == len(msgs)
    assert orbit._lib.orbit_strerror(-12).decode() == "unknown status"


def test_pattern_counts_and_noalloc_capacity():
    """Host-only calls: patterns with 2..k vertices (the oracle's tables)
    and the size of the static buffer of the allocation-free entry."""
    from paper_1911_10616_amd import orbit
    t = oracle.tables()
    k_of = [int(k) for k in t["pattern_k"]]
    for k in (3, 4, 5):
        assert orbit._lib.orbit_num_patterns(k) == sum(1 for x in k_of if 2 <= x <= k)
    assert orbit._lib.orbit_num_patterns(6) == 0
    orbit._lib.orbit_noalloc_capacity.restype = ctypes.c_uint64
    assert orbit._lib.orbit_noalloc_capacity() == 64 << 20


def test_bench_refuses_several_gpus():
    """bench.py counts on one GPU; asked for more it says so and fails."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
