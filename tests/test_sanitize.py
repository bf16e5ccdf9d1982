"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc -fsanitize=address,undefined, every report fatal), run through a small
C driver on a few graphs: no report, and the same counts as the ordinary
build -- induced, non-induced, edge orbits, and budget-limited rooted
enumeration (the cut-off path)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1911_10616_amd import graphgen as gg

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def asan_driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_asan")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fopenmp", "-pthread",
                           os.path.join(HERE, "sanitize_oracle_main.c"),
                           os.path.join(ROOT, "oracle", "orbit_oracle.c"), "-o", exe])
    return exe


def _graphs():
    return [gg.erdos_renyi(24, 0.3, 901), gg.barabasi_albert(30, 3, 902), gg.complete(7),
            gg.star(9), gg.erdos_renyi(1, 0.5, 903)]


@pytest.mark.parametrize("gi", range(5))
def test_oracle_clean_under_sanitizers(asan_driver, tmp_path, gi):
    rp, ci = _graphs()[gi]
    rp = np.asarray(rp, np.uint32)
    ci = np.asarray(ci, np.uint32)
    n = len(rp) - 1
    gpath, opath = str(tmp_path / "g.bin"), str(tmp_path / "o.bin")
    with open(gpath, "wb") as f:
        f.write(np.uint32(n).tobytes() + rp.tobytes() + ci.tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([asan_driver, gpath, opath], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    raw = np.fromfile(opath, dtype=np.uint8)
    rows, erows = n * 73, int(rp[-1]) * 12
    w = raw[: 8 * (3 * rows + erows)].view(np.uint64)
    ind, non = w[:rows].reshape(n, 73), w[rows:2 * rows].reshape(n, 73)
    edg = w[2 * rows:2 * rows + erows].reshape(-1, 12)
    root = w[2 * rows + erows:].reshape(n, 73)
    done = raw[8 * (3 * rows + erows):].astype(bool)
    np.testing.assert_array_equal(ind, oracle.induced_counts(rp, ci))
    np.testing.assert_array_equal(non, oracle.noninduced_counts(rp, ci))
    np.testing.assert_array_equal(edg, oracle.edge_counts(rp, ci).reshape(-1, 12))
    r2, d2 = oracle.rooted_counts(rp, ci, np.arange(n), kmax=5, budget=50)
    np.testing.assert_array_equal(root, r2)
    np.testing.assert_array_equal(done, d2)
    # rooted rows that finished within the budget are the full counts
    np.testing.assert_array_equal(root[done], ind[done])
