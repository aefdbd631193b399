"""Accuracy measures used by the tests and the benchmark.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``orthogonality``: max |Q^T Q - I| (columns).
* ``paper_orthogonality``: ||I - Q Q^T||_max, the paper's Example 2 measure.
* ``residual``: ||T Q - Q diag(lam)||_F / (n ||T||), ||T|| := max |lam|.
* ``eig_error``: max |lam - lam_ref| / ||T||.
* ``paper_residual``: ||A - Q Lambda Q^T||_c / ||A||_2, ||X||_c the largest
  column 2-norm (the paper's Example 3 measure).
"""

import numpy as np


def tridiag_matvec(d, e, X):
    """T(d, e) @ X without forming T."""
    Y = d[:, None] * X
    if d.shape[0] > 1:
        Y[:-1] += e[:, None] * X[1:]
        Y[1:] += e[:, None] * X[:-1]
    return Y


def orthogonality(Q):
    n = Q.shape[1]
    return float(np.abs(Q.T @ Q - np.eye(n)).max()) if n else 0.0


def residual(d, e, lam, Q):
    n = d.shape[0]
    if n == 0:
        return 0.0
    R = tridiag_matvec(np.asarray(d), np.asarray(e), Q) - Q * lam[None, :]
    tn = float(np.abs(lam).max()) or 1.0
    return float(np.linalg.norm(R) / (n * tn))


def eig_error(lam, lam_ref):
    tn = float(np.abs(lam_ref).max()) or 1.0
    return float(np.abs(np.asarray(lam) - np.asarray(lam_ref)).max() / tn)


def paper_residual(d, e, lam, Q):
    """||A - Q Lambda Q^T||_c / ||A||_2 (the paper's Example 3 measure), with
    ||X||_c the largest column 2-norm and ||A||_2 the spectral norm of the
    tridiagonal A = T(d, e), both formed densely (small n only)."""
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    A = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    R = A - (Q * np.asarray(lam)[None, :]) @ Q.T
    col = np.sqrt((R * R).sum(axis=0)).max()
    return float(col / (np.linalg.norm(A, 2) or 1.0))


def paper_orthogonality(Q):
    """||I - Q Q^T||_max (the paper's Example 2 measure; rows, not columns)."""
    n = Q.shape[0]
    return float(np.abs(Q @ Q.T - np.eye(n)).max()) if n else 0.0
