"""Plain FP64 Cuppen / Gu-Eisenstat divide and conquer (the oracle's solver).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows Algorithm 1 (and Algorithm 3 for the low-rank switch) of the paper:

1. T(d, e) with T[i, i+1] = T[i+1, i] = e[i] (eq. t, read with its sub-
   diagonal index garble fixed).
2. Blocks of at most ``leaf`` rows are solved by tridiagonal QR.
3. Otherwise tear at k = m // 2 (eq. T2): T = diag(T1, T2) + b_k v v^T.  With
   rho = |b_k| and sigma = sign(b_k) (+1 for b_k = 0) this is
   diag(T1', T2') + rho w w^T with w = e_k + sigma e_{k+1}, where T1' and T2'
   have rho subtracted from their corner diagonal entries.
4. Recurse on both halves, giving (Lambda_i, Q_i).
5. u = [last row of Q1, sigma * first row of Q2] (eq. T3); since ||u||^2 = 2
   we use z = u / sqrt(2) and rho' = 2 rho, so M = D + rho' z z^T
   (eq. rankone) with D = [Lambda_1; Lambda_2].
6. Deflation (section "Parallel Structured DC Algorithm", eq. T3-def and
   eq. evect): sort D stably; drop every i with rho'|z_i| <= tol; then walk
   the survivors in order and, when two neighbours p < i satisfy
   |(D_i - D_p) c s| <= tol for the Givens pair (c, s) = (z_i, z_p)/r that
   zeroes z_p, rotate their columns, update both D values and deflate p.
   tol = 8 eps max(max|D|, rho').
7. Secular roots, Loewner zhat and column scale (``oracle.secular``).
8. Q_new = [Q_nd U | deflated columns] (eq. updateV / eq. evect), with the
   new eigenvalues sorted ascending and the columns permuted with them.
9. Low-rank variant (Algorithm 3 with PSMMA via SRRSC): when the deflated
   size K reaches ``lr_min_k``, U is replaced by its block approximation from
   ``oracle.srrsc.lowrank_cauchy`` before the product.
"""

import math

import numpy as np

from . import leaf as _leaf
from . import secular as _sec
from . import srrsc as _srrsc

EPS = np.finfo(np.float64).eps


class MergeLog:
    """Per-merge record (size, deflated size, path) for tests and reports."""

    def __init__(self):
        self.records = []

    def add(self, **kw):
        self.records.append(kw)


def tear(d, e, k):
    """Split T(d, e) at row k (0-based rows [0, k) and [k, m)).

    Returns (d1, e1, d2, e2, rho, sigma) per eq. T2 with the corner
    corrections of step 3 in the module docstring.
    """
    b = float(e[k - 1])
    rho = abs(b)
    sigma = -1.0 if b < 0.0 else 1.0
    d1 = np.array(d[:k], dtype=np.float64)
    d2 = np.array(d[k:], dtype=np.float64)
    d1[-1] -= rho
    d2[0] -= rho
    return d1, np.array(e[:k - 1]), d2, np.array(e[k:]), rho, sigma


def deflate(D, z, rho2, Q):
    """Deflation of M = D + rho2 z z^T with eigenvector basis Q (m x m).

    Returns a dict: ``Dbar``/``zbar`` (K survivors, ascending), ``Qnd``
    (m x K columns of the rotated, sorted basis), ``Dd``/``Qd`` (deflated
    eigenpairs), ``nrot`` (number of pair rotations), ``tol``.
    """
    m = D.shape[0]
    order = np.argsort(D, kind="stable")
    Ds = D[order].copy()
    zs = z[order].copy()
    Qs = Q[:, order].copy()
    tol = 8.0 * EPS * max(float(np.abs(Ds).max()) if m else 0.0, rho2)
    defl = rho2 * np.abs(zs) <= tol
    keep = np.zeros(m, dtype=bool)
    nrot = 0
    p = -1
    for i in range(m):
        if defl[i]:
            continue
        if p < 0:
            p = i
            continue
        r = math.hypot(zs[p], zs[i])
        c = zs[i] / r
        s = zs[p] / r
        if abs((Ds[i] - Ds[p]) * c * s) <= tol:
            qp = Qs[:, p].copy()
            qi = Qs[:, i].copy()
            Qs[:, p] = c * qp - s * qi
            Qs[:, i] = s * qp + c * qi
            dp, di = Ds[p], Ds[i]
            Ds[p] = c * c * dp + s * s * di
            Ds[i] = s * s * dp + c * c * di
            zs[p] = 0.0
            zs[i] = r
            defl[p] = True
            nrot += 1
        else:
            keep[p] = True
        p = i
    if p >= 0:
        keep[p] = True
    return {
        "Dbar": Ds[keep], "zbar": zs[keep], "Qnd": Qs[:, keep],
        "Dd": Ds[~keep], "Qd": Qs[:, ~keep], "nrot": nrot, "tol": tol,
    }


def merge(lam1, Q1, lam2, Q2, rho, sigma, lr_tol=0.0, lr_block=512,
          lr_min_k=0, method="interp", log=None):
    """One merge (steps 5-9 of the module docstring)."""
    n1, n2 = lam1.shape[0], lam2.shape[0]
    m = n1 + n2
    D = np.concatenate([lam1, lam2])
    z = np.concatenate([Q1[-1, :], sigma * Q2[0, :]]) / math.sqrt(2.0)
    rho2 = 2.0 * rho
    Q = np.zeros((m, m))
    Q[:n1, :n1] = Q1
    Q[n1:, n1:] = Q2
    df = deflate(D, z, rho2, Q)
    Dbar, zbar = df["Dbar"], df["zbar"]
    K = Dbar.shape[0]
    path = "none"
    ranks = None
    if K > 0:
        org, tau, zhat, s = _sec.solve_rank_one(Dbar, zbar, rho2, method=method)
        lam_new = Dbar[org] + tau
        if lr_tol > 0.0 and K >= lr_min_k and K > lr_block:
            U, ranks = _srrsc.lowrank_cauchy(Dbar, org, tau, zhat, s,
                                             lr_tol, lr_block)
            path = "lowrank"
        else:
            U = _sec.cauchy_matrix(Dbar, org, tau, zhat, s)
            path = "plain"
        C = df["Qnd"] @ U
    else:
        lam_new = np.empty(0)
        C = np.empty((m, 0))
    lam = np.concatenate([lam_new, df["Dd"]])
    Qm = np.concatenate([C, df["Qd"]], axis=1)
    order = np.argsort(lam, kind="stable")
    if log is not None:
        log.add(m=m, K=K, nrot=df["nrot"], path=path, ranks=ranks)
    return lam[order], Qm[:, order]


def eigh_tridiagonal(d, e, leaf=32, lr_tol=0.0, lr_block=512, lr_min_k=0,
                     method="interp", log=None):
    """All eigenpairs of T(d, e) by divide and conquer (Algorithm 1 / 3).

    Returns (lam ascending, Q) with T = Q diag(lam) Q^T.
    """
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    n = d.shape[0]
    if n == 0:
        return np.empty(0), np.empty((0, 0))
    if n <= max(leaf, 1):
        return _leaf.tridiag_qr(d, e)
    k = n // 2
    d1, e1, d2, e2, rho, sigma = tear(d, e, k)
    lam1, Q1 = eigh_tridiagonal(d1, e1, leaf, lr_tol, lr_block, lr_min_k,
                                method, log)
    lam2, Q2 = eigh_tridiagonal(d2, e2, leaf, lr_tol, lr_block, lr_min_k,
                                method, log)
    return merge(lam1, Q1, lam2, Q2, rho, sigma, lr_tol, lr_block, lr_min_k,
                 method, log)
