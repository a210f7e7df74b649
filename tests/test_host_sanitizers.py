"""The host analysis (ordering, symbolic factorization, maps: ordering.cpp and
symbolic.cpp) built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer
and run on patterns of every kind the library meets -- tight-binding supercells,
FEM grids, a random symmetric pattern, a single vertex, disconnected blocks, a
dense block, an unsymmetric pattern (rejected) -- with the structural invariants
of the result checked by the driver, and its statistics equal to those of the
library's own build (kth_analyze)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import pencilgen as pg

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1710_05134_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("asan") / "host_analysis")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", CSRC,
           os.path.join(HERE, "host_analysis_driver.cpp"), os.path.join(CSRC, "ordering.cpp"),
           os.path.join(CSRC, "symbolic.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


def _csr_from_edges(n, edges):
    rows = [set([i]) for i in range(n)]
    for i, j in edges:
        rows[i].add(j)
        rows[j].add(i)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    cols = []
    for i in range(n):
        c = sorted(rows[i])
        cols.extend(c)
        rowptr[i + 1] = rowptr[i] + len(c)
    return rowptr, np.array(cols, dtype=np.int32)


def _patterns():
    out = {}
    for name, p in [("tiny", pg.workload("tiny")), ("tb444", pg.tb_supercell((4, 4, 4), seed=1)),
                    ("tb886", pg.tb_supercell((8, 8, 6), seed=2)),
                    ("fem", pg.fem_tensor((9, 10, 11), (1.0, 1.3, 0.7)))]:
        out[name] = (p.rowptr, p.col)
    rng = np.random.default_rng(5)
    n = 3000
    e = rng.integers(0, n, size=(4 * n, 2))
    out["random"] = _csr_from_edges(n, [(int(a), int(b)) for a, b in e if a != b])
    out["single"] = _csr_from_edges(1, [])
    out["blocks"] = _csr_from_edges(40, [(i, i + 1) for i in range(0, 39) if i % 10 != 9])
    out["dense"] = _csr_from_edges(64, [(i, j) for i in range(64) for j in range(i + 1, 64)])
    return out


def _write(path, rowptr, col):
    n = len(rowptr) - 1
    with open(path, "wb") as f:
        f.write(np.int64(n).tobytes())
        f.write(np.int64(len(col)).tobytes())
        f.write(np.ascontiguousarray(rowptr, dtype=np.int64).tobytes())
        f.write(np.ascontiguousarray(col, dtype=np.int32).tobytes())


def _run(driver, path):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return subprocess.run([driver, path], capture_output=True, text=True, timeout=600, env=env)


@pytest.mark.parametrize("name", ["tiny", "tb444", "tb886", "fem", "random", "single", "blocks",
                                  "dense"])
def test_analysis_clean_under_sanitizers(driver, tmp_path, name):
    rowptr, col = _patterns()[name]
    path = str(tmp_path / f"{name}.bin")
    _write(path, rowptr, col)
    r = _run(driver, path)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    nsup, flops, nnz_l, max_front, nlevels = r.stdout.split()
    import paper_1710_05134_amd as K
    a = K.kth_analyze(rowptr, col)
    assert int(nsup) == int(a["n_supernodes"])
    assert float(flops) == a["flops"]
    assert int(nnz_l) == int(a["nnz_l"])
    assert int(max_front) == int(a["max_front"])


def test_unsymmetric_pattern_rejected(driver, tmp_path):
    rowptr = np.array([0, 2, 3], dtype=np.int64)
    col = np.array([0, 1, 1], dtype=np.int32)   # (0, 1) without (1, 0)
    path = str(tmp_path / "unsym.bin")
    _write(path, rowptr, col)
    r = _run(driver, path)
    assert r.returncode == 0 and r.stdout.startswith("rejected"), (r.stdout, r.stderr[-2000:])
