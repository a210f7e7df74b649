"""CPU-side checks of the C ABI library (no GPU needed).

* libkth.so loads and exports every function include/kth.h declares;
* the host analysis (nested dissection, symbolic factorization) returns a valid
  permutation and counts consistent with an independent count from the oracle
  side's structure rules;
* malformed patterns are rejected with KTH_EINVAL;
* without a GPU, creating a context fails with KTH_EDEVICE instead of crashing.
"""
import os
import re
import subprocess

import numpy as np
import pytest

import pencilgen as pg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kth.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kth_[a-z_0-9]+)\s*\(", src)) - {"kth_alloc_fn", "kth_free_fn"})


def test_library_exports_every_declared_symbol():
    import paper_1710_05134_amd as K
    K.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", K.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    decl = declared_functions()
    assert len(decl) >= 20
    missing = [d for d in decl if d not in exported]
    assert not missing, missing


def test_analysis_permutation_and_counts():
    import paper_1710_05134_amd as K
    for p in (pg.tb_supercell((3, 3, 2), seed=1), pg.fem_tensor((6, 5, 7)), pg.chain(50),
              pg.block_diag_perm((9, 4, 12), seed=2)):
        st, perm = K.kth_analyze(p.rowptr, p.col, check_symmetry=True, want_perm=True)
        assert sorted(perm.tolist()) == list(range(p.n))
        assert st["n"] == p.n and st["nnz"] == p.nnz
        assert st["flops_padded"] >= st["flops"] > 0 or p.n == 1
        assert st["nnz_l_padded"] >= st["nnz_l"]
        # column counts of L under the library's order, by a plain dense symbolic
        # elimination (fill of the permuted pattern) -- independent of its code
        A = np.zeros((p.n, p.n), dtype=bool)          # the stored pattern (explicit zeros count)
        A[np.repeat(np.arange(p.n), np.diff(p.rowptr)), p.col] = True
        Ap = A[np.ix_(perm, perm)]
        n = p.n
        S = Ap.copy()
        flops = 0.0
        nnzl = 0
        for j in range(n):
            rows = np.nonzero(S[j + 1:, j])[0] + j + 1
            c = rows.size
            nnzl += c
            flops += c * c + 2 * c
            S[np.ix_(rows, rows)] = True
        assert nnzl == st["nnz_l"]
        assert flops == st["flops"]


def test_analysis_supervariables_tb():
    import paper_1710_05134_amd as K
    p = pg.tb_supercell((2, 2, 2))
    st = K.kth_analyze(p.rowptr, p.col)
    assert st["n_supervariables"] == p.n // 4   # the four orbitals of an atom


@pytest.mark.parametrize("case", ["unsorted", "out_of_range", "no_diagonal", "asymmetric"])
def test_bad_patterns_rejected(case):
    import paper_1710_05134_amd as K
    p = pg.chain(10)
    rowptr, col = p.rowptr.copy(), p.col.copy()
    if case == "unsorted":
        col[1], col[2] = col[2], col[1]
    elif case == "out_of_range":
        col[-1] = 99
    elif case == "no_diagonal":
        rowptr = np.array([0, 1, 2], dtype=np.int64)
        col = np.array([1, 0], dtype=np.int32)
    elif case == "asymmetric":
        rowptr = np.array([0, 2, 3], dtype=np.int64)
        col = np.array([0, 1, 1], dtype=np.int32)
    with pytest.raises(K.KthError) as e:
        K.kth_analyze(rowptr, col, check_symmetry=True)
    assert e.value.status == K.KTH_EINVAL


def test_context_without_gpu_fails_cleanly():
    import torch
    import paper_1710_05134_amd as K
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(K.KthError) as e:
        K.Context(0)
    assert e.value.status == K.KTH_EDEVICE
