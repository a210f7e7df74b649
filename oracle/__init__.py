"""CPU oracle for the k-th eigenpair method (test infrastructure only).

Plain, slow, obviously-correct reference implementations used to check the
GPU library: nothing in the product library imports, links or calls this
package.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` use it.

* ``oracle.dense``   dense path: Cholesky reduction of the pencil and a
  symmetric eigensolver (the route of LAPACK's generalized solver used as the
  comparison in Section 4.2); nu(sigma) by counting eigenvalues.
* ``oracle.sparse``  scalar multifrontal LDL^T of A - sigma B with restricted
  Bunch-Kaufman pivoting (Section 2.1, Section 3.3) in plain C, inertia and solves.
* ``oracle.three_stage``  Alg. 2 -> Alg. 1' -> Alg. 3 (Alg. 4) in FP64 over the
  sparse oracle.
* ``oracle.ordering`` coordinate nested dissection used as the oracle's Q.
"""
