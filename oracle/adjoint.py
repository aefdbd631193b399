"""Dense reverse-mode gradient of the tridiagonal eigendecomposition.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

For T = Q diag(lam) Q^T with distinct eigenvalues and a loss L(lam, Q) with
cotangents (lam_bar, Q_bar), the cotangent of the matrix is (Giles 2008,
"Collected matrix derivative results for forward and reverse mode AD")

    A_bar = Q (diag(lam_bar) + F o (Q^T Q_bar)) Q^T,
    F_ij = 1 / (lam_j - lam_i) for i != j,  F_ii = 0.

T depends on d_i through T[i, i] and on e_i through both T[i, i+1] and
T[i+1, i], hence d_bar_i = A_bar[i, i] and e_bar_i = A_bar[i, i+1] +
A_bar[i+1, i].  Written out densely, with no band-only shortcut.
"""

import numpy as np


def backward(lam, Q, lam_bar=None, Q_bar=None):
    lam = np.asarray(lam, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    n = lam.shape[0]
    M = np.zeros((n, n))
    if lam_bar is not None:
        M += np.diag(np.asarray(lam_bar, dtype=np.float64))
    if Q_bar is not None:
        G = Q.T @ np.asarray(Q_bar, dtype=np.float64)
        diff = lam[None, :] - lam[:, None]          # lam_j - lam_i
        with np.errstate(divide="ignore"):
            F = np.where(diff != 0.0, 1.0 / np.where(diff != 0.0, diff, 1.0), 0.0)
        np.fill_diagonal(F, 0.0)
        M += F * G
    A_bar = Q @ M @ Q.T
    d_bar = np.diag(A_bar).copy()
    e_bar = np.diag(A_bar, 1) + np.diag(A_bar, -1)
    return d_bar, e_bar
