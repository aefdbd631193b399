"""CPU oracle for the structured divide-and-conquer tridiagonal eigensolver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 NumPy
implementation of what the GPU path computes.  It exists so that tests, the
package's smoke check and the benchmark's CPU-baseline leg can compare the
HIP path against an independent result.  Nothing in the product path may
import it, and it imports nothing from the product package.

Modules (each function cites the passage of Liao, Li, Lu and Roman, "A
parallel structured divide-and-conquer algorithm for symmetric tridiagonal
eigenvalue problems", IEEE TPDS 2020, that it follows):

* ``leaf``     -- tridiagonal QR with Wilkinson shift for small blocks
                  (Algorithm 1, "apply the QR algorithm").
* ``secular``  -- secular roots, Loewner recomputation of z, column scale and
                  the Cauchy-like eigenvector matrix (eq. secular,
                  eq. eigenvector, eq. Q_Cauchy, Remark 3 eq. d-lambda).
* ``dc``       -- the recursion: tear (eq. T2/T3), deflation (section
                  "Parallel Structured DC Algorithm", eq. T3-def / evect),
                  merge update (eq. updateV), plain and low-rank variants.
* ``srrsc``    -- structured low-rank compression of Cauchy-like blocks
                  (section "SRRSC low-rank approximation", Theorems 1-2,
                  eq. sid, eq. geneZ).
* ``adjoint``  -- dense reverse-mode gradient of (lambda, Q) w.r.t. (d, e).
* ``sturm``    -- Sturm-sequence bisection (independent eigenvalue pin).
* ``metrics``  -- orthogonality / residual / eigenvalue-error measures.

Parity pins for every function live in ``tests/test_oracle_*.py``.
"""

from . import leaf, secular, dc, srrsc, adjoint, sturm, metrics  # noqa: F401
