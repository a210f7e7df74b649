"""Seeded synthetic pencils (A, B) and start vectors.

This module only *builds inputs*: it holds none of the eigen-method's
arithmetic, so both the GPU library and the CPU oracle can draw from it.

Pencils produced here
---------------------
* ``tb_supercell``  periodic diamond-lattice tight-binding pencil, 4 orbitals per
  atom, nearest-neighbour 4x4 blocks.  It stands in for the electronic-structure
  pencils of the paper's Table 1 (which are not available): A real symmetric,
  B symmetric positive definite with unit diagonal (Appendix A: normalised
  basis functions give diag(B) = 1), A and B on one sparsity pattern
  (Section 4.1), k = n/2 (highest occupied state, Appendix B).
* ``tb_cluster``    the same value laws on an open-boundary ball-carved cluster of
  any atom count (used for many uneven small pencils).
* ``fem_tensor``    3-D tensor-product linear-FEM Laplacian pencil with a
  non-diagonal SPD mass matrix; its spectrum is known in closed form, so it pins
  inertia counts at any size.
* ``block_diag_perm`` randomly permuted block-diagonal pencil (exact spectrum from
  the blocks).
* ``chain``         tridiagonal Toeplitz A with B = I (the Sturm / Givens case).

All matrices are returned in CSR with both triangles stored, int64 row
pointers, int32 sorted column indices and float64 values, A and B sharing
one pattern.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

# diamond conventional cell, carbon
A_LATT = 3.567                     # angstrom
BOND0 = A_LATT * math.sqrt(3.0) / 4.0   # ideal bond length d0 = r0 = 1.5446 angstrom
# 8-atom basis of the conventional cell, in units of a/4; first four are sublattice A
_BASIS = np.array([(0, 0, 0), (0, 2, 2), (2, 0, 2), (2, 2, 0),
                   (1, 1, 1), (1, 3, 3), (3, 1, 3), (3, 3, 1)], dtype=np.int64)
# nearest-neighbour offsets of an A-sublattice atom (units of a/4)
_OFFS = np.array([(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)], dtype=np.int64)
NORB = 4


@dataclasses.dataclass
class Pencil:
    n: int
    rowptr: np.ndarray      # int64[n+1]
    col: np.ndarray         # int32[nnz]
    a_val: np.ndarray       # float64[nnz]
    b_val: np.ndarray       # float64[nnz]
    coords: np.ndarray | None = None   # float64[n, 3] position of each dof (atom centre)
    k: int | None = None
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def A(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.a_val, self.col, self.rowptr), shape=(self.n, self.n))

    def B(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.b_val, self.col, self.rowptr), shape=(self.n, self.n))


def _csr_from_blocks(n: int, rows: np.ndarray, cols: np.ndarray,
                     av: np.ndarray, bv: np.ndarray) -> tuple:
    """Assemble COO triplets (no duplicates allowed) into sorted CSR arrays."""
    order = np.lexsort((cols, rows))
    rows, cols, av, bv = rows[order], cols[order], av[order], bv[order]
    if rows.size > 1:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if dup.any():
            raise ValueError("duplicate entries in pencil construction")
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int64)
    return rowptr, cols.astype(np.int32), av.astype(np.float64), bv.astype(np.float64)


def _tb_values_from_bonds(rng, natoms, onsite, bond_i, bond_j, r):
    """Values of the TB pencil given bonds (i<->j) and bond lengths.  The random
    draws happen in the documented order: on-site, A blocks, B blocks."""
    n = natoms * NORB
    nb = bond_i.size
    hblk = rng.normal(0.0, 1.5, size=(nb, NORB, NORB)) * np.exp(-r / BOND0)[:, None, None]
    sblk = rng.normal(0.0, 0.03, size=(nb, NORB, NORB))
    o = np.arange(NORB)
    # on-site 4x4 blocks: A diagonal = onsite, off-diagonals explicit zeros; B = I
    at = np.repeat(np.arange(natoms), NORB * NORB)
    oi = np.tile(np.repeat(o, NORB), natoms)
    oj = np.tile(np.tile(o, NORB), natoms)
    r_on = at * NORB + oi
    c_on = at * NORB + oj
    a_on = np.where(oi == oj, onsite.reshape(-1)[at * NORB + oi], 0.0)
    b_on = np.where(oi == oj, 1.0, 0.0)
    # bond blocks: A[i,j] = H, A[j,i] = H^T (mirrored), same for B
    bi = np.repeat(bond_i, NORB * NORB)
    bj = np.repeat(bond_j, NORB * NORB)
    pi = np.tile(np.repeat(o, NORB), nb)
    pj = np.tile(np.tile(o, NORB), nb)
    hv = hblk.reshape(-1)
    sv = sblk.reshape(-1)
    rows = np.concatenate([r_on, bi * NORB + pi, bj * NORB + pj])
    cols = np.concatenate([c_on, bj * NORB + pj, bi * NORB + pi])
    av = np.concatenate([a_on, hv, hv])
    bv = np.concatenate([b_on, sv, sv])
    return _csr_from_blocks(n, rows, cols, av, bv)


def tb_supercell(cells=(4, 4, 4), seed: int = 0, k: int | None = None) -> Pencil:
    """Periodic diamond supercell of Lx*Ly*Lz conventional cells (8 atoms each).

    Atom index = ((ix*Ly + iy)*Lz + iz)*8 + basis.  Draw order with
    ``numpy.random.default_rng(seed)``: jitter U(-0.05, 0.05) angstrom per
    coordinate, on-site energies U(-8, 2) eV per orbital, A bond blocks
    N(0, 1.5) * exp(-r/r0), B bond blocks N(0, 0.03); bonds ordered by
    (A-atom index, offset index); r is the jittered minimum-image bond length.
    """
    Lx, Ly, Lz = (int(c) for c in cells)
    rng = np.random.default_rng(seed)
    ix, iy, iz, b = np.meshgrid(np.arange(Lx), np.arange(Ly), np.arange(Lz), np.arange(8),
                                indexing="ij")
    ix, iy, iz, b = ix.ravel(), iy.ravel(), iz.ravel(), b.ravel()
    natoms = ix.size
    icoord = np.stack([4 * ix, 4 * iy, 4 * iz], axis=1) + _BASIS[b]   # units of a/4
    jitter = rng.uniform(-0.05, 0.05, size=(natoms, 3))
    onsite = rng.uniform(-8.0, 2.0, size=(natoms, NORB))
    # lookup (integer coords -> atom index)
    dims = np.array([4 * Lx, 4 * Ly, 4 * Lz], dtype=np.int64)
    key_of = lambda c: (c[:, 0] * dims[1] + c[:, 1]) * dims[2] + c[:, 2]
    lut = -np.ones(int(dims.prod()), dtype=np.int64)
    lut[key_of(icoord)] = np.arange(natoms)
    a_atoms = np.nonzero(b < 4)[0]
    bond_i = np.repeat(a_atoms, 4)
    off = np.tile(_OFFS, (a_atoms.size, 1))
    nbr = (icoord[bond_i] + off) % dims
    bond_j = lut[key_of(nbr)]
    if (bond_j < 0).any():
        raise RuntimeError("lattice neighbour lookup failed")
    d = off * (A_LATT / 4.0) + jitter[bond_j] - jitter[bond_i]
    r = np.sqrt((d * d).sum(axis=1))
    rowptr, col, av, bv = _tb_values_from_bonds(rng, natoms, onsite, bond_i, bond_j, r)
    pos = icoord * (A_LATT / 4.0) + jitter
    n = natoms * NORB
    return Pencil(n=n, rowptr=rowptr, col=col, a_val=av, b_val=bv,
                  coords=np.repeat(pos, NORB, axis=0), k=(n // 2 if k is None else k),
                  name=f"tb{Lx}x{Ly}x{Lz}")


def tb_cluster(natoms: int, seed=0, k: int | None = None) -> Pencil:
    """Open-boundary cluster of the ``natoms`` ideal diamond sites nearest the
    origin (ties broken lexicographically on integer coordinates), then the
    same jitter / value laws as ``tb_supercell`` (draw order identical).
    ``seed`` may be an int or a ``numpy.random.SeedSequence``."""
    rng = np.random.default_rng(seed)
    R = int(math.ceil((natoms * 3.0 / (4.0 * math.pi) * 8.0 / 64.0) ** (1.0 / 3.0) * 4)) + 6
    g = np.arange(-R, R + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    c = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    m = c % 4
    isA = ((m[:, 0] % 2 == 0) & (m[:, 1] % 2 == 0) & (m[:, 2] % 2 == 0)
           & (((m[:, 0] + m[:, 1] + m[:, 2]) // 2) % 2 == 0))
    isB = ((m[:, 0] % 2 == 1) & (m[:, 1] % 2 == 1) & (m[:, 2] % 2 == 1)
           & ((((m[:, 0] - 1) + (m[:, 1] - 1) + (m[:, 2] - 1)) // 2) % 2 == 0))
    sel = isA | isB
    c, isA = c[sel], isA[sel]
    r2 = (c * c).sum(axis=1)
    order = np.lexsort((c[:, 2], c[:, 1], c[:, 0], r2))
    if order.size < natoms:
        raise RuntimeError("cluster radius too small")
    c, isA = c[order[:natoms]], isA[order[:natoms]]
    jitter = rng.uniform(-0.05, 0.05, size=(natoms, 3))
    onsite = rng.uniform(-8.0, 2.0, size=(natoms, NORB))
    lut = {tuple(v): i for i, v in enumerate(c.tolist())}
    bi, bj, offs = [], [], []
    for i in np.nonzero(isA)[0].tolist():
        for o in _OFFS.tolist():
            j = lut.get((c[i, 0] + o[0], c[i, 1] + o[1], c[i, 2] + o[2]))
            if j is not None:
                bi.append(i); bj.append(j); offs.append(o)
    bond_i = np.array(bi, dtype=np.int64)
    bond_j = np.array(bj, dtype=np.int64)
    off = np.array(offs, dtype=np.int64).reshape(-1, 3)
    d = off * (A_LATT / 4.0) + jitter[bond_j] - jitter[bond_i]
    r = np.sqrt((d * d).sum(axis=1))
    rowptr, col, av, bv = _tb_values_from_bonds(rng, natoms, onsite, bond_i, bond_j, r)
    n = natoms * NORB
    pos = c * (A_LATT / 4.0) + jitter
    return Pencil(n=n, rowptr=rowptr, col=col, a_val=av, b_val=bv,
                  coords=np.repeat(pos, NORB, axis=0), k=(n // 2 if k is None else k),
                  name=f"cluster{natoms}")


def uneven_batch(count=256, seed=0, n_lo=500, n_hi=8000):
    """``count`` clusters with n_target ~ U{n_lo..n_hi}, atoms = n_target // 4,
    k ~ U{floor(0.3 n)..floor(0.5 n)}; pencil i seeded with SeedSequence(seed).spawn(count)[i]."""
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(count)
    top = np.random.default_rng(np.random.SeedSequence(seed, spawn_key=(10**6,)))
    ntar = top.integers(n_lo, n_hi + 1, size=count)
    out = []
    for i in range(count):
        na = max(int(ntar[i]) // NORB, 2)
        r = np.random.default_rng(kids[i].spawn(1)[0])
        n = na * NORB
        k = int(r.integers(int(0.3 * n), int(0.5 * n) + 1))
        out.append(tb_cluster(na, seed=kids[i], k=k))
    return out


def fem_tensor(N=(6, 7, 8), w=(1.0, 1.3, 1.7), k: int | None = None) -> Pencil:
    """Q1-free tensor-product linear FEM pencil on the unit cube, Dirichlet BC.

    K_d = w_d * tridiag(-1, 2, -1) / h_d, M_d = (h_d / 6) tridiag(1, 4, 1),
    h_d = 1 / (N_d + 1); A = Kx(x)My(x)Mz + Mx(x)Ky(x)Mz + Mx(x)My(x)Kz, B = Mx(x)My(x)Mz.
    The 27-point pattern of A and B coincide.  dof index = (i*Ny + j)*Nz + l.
    """
    mats = []
    for Nd, wd in zip(N, w):
        h = 1.0 / (Nd + 1)
        e = np.ones(Nd)
        K = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1]) * (wd / h)
        M = sp.diags([e[:-1], 4 * e, e[:-1]], [-1, 0, 1]) * (h / 6.0)
        mats.append((sp.csr_matrix(K), sp.csr_matrix(M)))
    (Kx, Mx), (Ky, My), (Kz, Mz) = mats
    kron = lambda a, b, c: sp.kron(sp.kron(a, b), c, format="csr")
    A = kron(Kx, My, Mz) + kron(Mx, Ky, Mz) + kron(Mx, My, Kz)
    B = kron(Mx, My, Mz)
    n = A.shape[0]
    # force one shared pattern (27-point stencil) with explicit zeros where needed
    P = (abs(A) + abs(B)).tocsr()
    P.sort_indices()
    A2 = _on_pattern(A, P)
    B2 = _on_pattern(B, P)
    ii, jj, ll = np.meshgrid(np.arange(N[0]), np.arange(N[1]), np.arange(N[2]), indexing="ij")
    coords = np.stack([ii.ravel(), jj.ravel(), ll.ravel()], axis=1).astype(np.float64)
    return Pencil(n=n, rowptr=P.indptr.astype(np.int64), col=P.indices.astype(np.int32),
                  a_val=A2, b_val=B2, coords=coords, k=(n // 2 if k is None else k),
                  name=f"fem{N[0]}x{N[1]}x{N[2]}")


def _on_pattern(M: sp.csr_matrix, P: sp.csr_matrix) -> np.ndarray:
    """Values of M on the (sorted) pattern of P (zeros where M has no entry)."""
    M = M.tocsr()
    M.sort_indices()
    out = np.zeros(P.nnz, dtype=np.float64)
    for r in range(P.shape[0]):
        a, b = P.indptr[r], P.indptr[r + 1]
        ma, mb = M.indptr[r], M.indptr[r + 1]
        pos = np.searchsorted(P.indices[a:b], M.indices[ma:mb])
        out[a + pos] = M.data[ma:mb]
    return out


def block_diag_perm(sizes=(5, 7, 3, 9), seed=0, k: int | None = None) -> Pencil:
    """Random dense symmetric blocks A_b and SPD blocks B_b, assembled block
    diagonally and then symmetrically permuted by a random permutation.
    Returns the pencil and (in ``.blocks``) the unpermuted blocks."""
    rng = np.random.default_rng(seed)
    blocks = []
    for s in sizes:
        X = rng.normal(size=(s, s))
        Ab = (X + X.T) / 2.0
        Y = rng.normal(size=(s, s)) * 0.2
        Bb = np.eye(s) + (Y @ Y.T) / s
        blocks.append((Ab, Bb))
    A = sp.block_diag([b[0] for b in blocks], format="csr")
    B = sp.block_diag([b[1] for b in blocks], format="csr")
    n = A.shape[0]
    p = rng.permutation(n)
    A = A[p][:, p].tocsr()
    B = B[p][:, p].tocsr()
    P = (abs(A) + abs(B) + sp.identity(n)).tocsr()
    P.sort_indices()
    pen = Pencil(n=n, rowptr=P.indptr.astype(np.int64), col=P.indices.astype(np.int32),
                 a_val=_on_pattern(A, P), b_val=_on_pattern(B, P),
                 k=(n // 2 if k is None else k), name="blockdiag")
    pen.blocks = blocks
    pen.perm = p
    return pen


def chain(n=64, a=0.5, b=-1.0, k: int | None = None) -> Pencil:
    """Tridiagonal Toeplitz A = tridiag(b, a, b), B = I."""
    e = np.ones(n)
    A = sp.diags([b * e[:-1], a * e, b * e[:-1]], [-1, 0, 1], format="csr")
    A.sort_indices()
    return Pencil(n=n, rowptr=A.indptr.astype(np.int64), col=A.indices.astype(np.int32),
                  a_val=A.data.astype(np.float64),
                  b_val=np.where(np.repeat(np.arange(n), np.diff(A.indptr)) == A.indices, 1.0, 0.0),
                  coords=np.stack([np.arange(n), np.zeros(n), np.zeros(n)], axis=1).astype(float),
                  k=(n // 2 if k is None else k), name=f"chain{n}")


def doubled(pen: Pencil, seed: int | None = 0, k: int | None = None) -> Pencil:
    """The direct sum of a pencil with itself, symmetrically permuted by a seeded
    random permutation (seed None: the two copies kept in blocks): every
    eigenvalue of ``pen`` becomes an exactly double one.  (A test input for
    multiple eigenvalues; no arithmetic on the values.)"""
    A = sp.block_diag([pen.A(), pen.A()], format="csr")
    B = sp.block_diag([pen.B(), pen.B()], format="csr")
    n = A.shape[0]
    perm = np.arange(n) if seed is None else np.random.default_rng(seed).permutation(n)
    A = A[perm][:, perm].tocsr()
    B = B[perm][:, perm].tocsr()
    A.sort_indices()
    B.sort_indices()
    P = (abs(A) + abs(B)).tocsr()
    P.sort_indices()
    out = Pencil(n=n, rowptr=P.indptr.astype(np.int64), col=P.indices.astype(np.int32),
                 a_val=_on_pattern(A, P), b_val=_on_pattern(B, P),
                 k=(n // 2 if k is None else k), name=f"doubled_{pen.name}")
    out.perm = perm
    return out


def start_vectors(n: int, seed: int = 0, count: int = 4) -> np.ndarray:
    """Random starting vectors (N(0,1) entries), shape (count, n).  Row 0 starts
    the stage-1 Lanczos process, row 1 the shift-and-invert Lanczos process,
    rows 2 and 3 serve restarts after a breakdown, rows 4.. the further columns of
    a block shift-and-invert start (column 0 is row 1).  The rows do not depend on
    ``count`` (the normals are drawn row after row).  Drawn from a child of
    SeedSequence(seed) kept apart from the pencil's own stream."""
    child = np.random.SeedSequence(seed).spawn(2)[1]
    return np.random.default_rng(child).standard_normal(size=(count, n))


# configurations of the workloads, by name
CONFIGS = {
    "tiny": dict(cells=(4, 4, 4)),           # n = 2048
    "n131k": dict(cells=(16, 16, 16)),       # n = 131072
    "n524k": dict(cells=(32, 32, 16)),       # n = 524288
    "n1_5m": dict(cells=(36, 36, 36)),       # n = 1492992
}


def workload(name: str, seed: int = 0) -> Pencil:
    return tb_supercell(CONFIGS[name]["cells"], seed=seed)
