"""Leaf eigensolver of the oracle: implicit symmetric tridiagonal QR.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Algorithm 1 of the paper solves a block that is "small enough" with the QR
algorithm.  This is the textbook implicit symmetric QR step with a Wilkinson
shift (Golub & Van Loan, "Matrix Computations", section 8.3), one Givens
rotation per bulge-chase position, accumulated into the eigenvector matrix.
"""

import math

import numpy as np

EPS = np.finfo(np.float64).eps


def _givens(x, y):
    """Return (c, s, r) with [c s; -s c] [x; y] = [r; 0]."""
    if y == 0.0:
        return 1.0, 0.0, x
    r = math.hypot(x, y)
    return x / r, y / r, r


def tridiag_qr(d, e, max_sweeps_per_eig=40):
    """Eigen-decomposition of the symmetric tridiagonal T(d, e).

    T[i, i] = d[i], T[i, i+1] = T[i+1, i] = e[i].  Returns (lam, Z) with lam
    ascending and T = Z diag(lam) Z^T, Z orthogonal.  Raises RuntimeError if a
    sub-diagonal entry fails to converge.
    """
    d = np.array(d, dtype=np.float64, copy=True)
    e = np.array(e, dtype=np.float64, copy=True)
    n = d.shape[0]
    Z = np.eye(n)
    if n == 0:
        return d, Z
    # Absolute deflation threshold eps * ||T||_inf: DC's eigenvalue accuracy is
    # absolute in ||T||, and a relative test would stall where d == 0.
    anorm = np.abs(d).copy()
    if n > 1:
        anorm[:-1] += np.abs(e)
        anorm[1:] += np.abs(e)
    thresh = EPS * float(anorm.max()) if anorm.max() > 0 else 0.0

    hi = n - 1
    sweeps = 0
    while hi > 0:
        if abs(e[hi - 1]) <= thresh:
            e[hi - 1] = 0.0
            hi -= 1
            sweeps = 0
            continue
        lo = hi - 1
        while lo > 0 and abs(e[lo - 1]) > thresh:
            lo -= 1
        if lo > 0:
            e[lo - 1] = 0.0
        sweeps += 1
        if sweeps > max_sweeps_per_eig:
            raise RuntimeError("tridiagonal QR did not converge")
        # Wilkinson shift from the trailing 2x2 block of the active window.
        delta = 0.5 * (d[hi - 1] - d[hi])
        b = e[hi - 1]
        sgn = 1.0 if delta >= 0.0 else -1.0
        mu = d[hi] - b * b / (delta + sgn * math.hypot(delta, b))
        x = d[lo] - mu
        y = e[lo]
        bulge = 0.0
        for k in range(lo, hi):
            if k > lo:
                x = e[k - 1]
                y = bulge
            c, s, r = _givens(x, y)
            if k > lo:
                e[k - 1] = r
            a, f, g = d[k], e[k], d[k + 1]
            # T <- G T G^T on rows/columns (k, k+1), G = [c s; -s c].
            d[k] = c * c * a + 2.0 * c * s * f + s * s * g
            d[k + 1] = s * s * a - 2.0 * c * s * f + c * c * g
            e[k] = c * s * (g - a) + (c * c - s * s) * f
            if k + 1 < hi:
                bulge = s * e[k + 1]
                e[k + 1] = c * e[k + 1]
            # Z <- Z G^T keeps T_original = Z T Z^T.
            zk = Z[:, k].copy()
            zk1 = Z[:, k + 1]
            Z[:, k] = c * zk + s * zk1
            Z[:, k + 1] = -s * zk + c * zk1
    order = np.argsort(d, kind="stable")
    return d[order], Z[:, order]
