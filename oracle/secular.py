"""Secular equation, Loewner recomputation and Cauchy-like eigenvectors.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The merge reduces to the eigenproblem of M = D + rho z z^T (eq. rankone) with
D = diag(D_1 < ... < D_K) and every z_i != 0 after deflation.  Its
eigenvalues are the roots of the secular function (eq. secular; the printed
formula lost its summation sign, restored here):

    f(lam) = 1 + rho * sum_i z_i^2 / (D_i - lam),

which interlace the poles, D_j < lam_j < D_{j+1}, the last one in
(D_K, D_K + rho ||z||^2].  Each root is stored as an origin index o_j and an
offset tau_j = lam_j - D_{o_j}, so every difference D_i - lam_j is formed as
(D_i - D_{o_j}) - tau_j and never by subtracting a stored lam_j (Remark 3,
eq. d-lambda, which keeps two distances gamma/mu; one nearest-pole offset
carries the same information).

The eigenvector of lam_j is (D - lam_j I)^{-1} z, normalised (eq. eigenvector);
all K of them form the Cauchy-like matrix of eq. Q_Cauchy,
U_ij = zhat_i s_j / (D_i - lam_j).  Following Gu and Eisenstat (1995) z is
first replaced by zhat, the vector for which the computed roots are exact
eigenvalues (Loewner's formula), which is what keeps U orthogonal to working
precision.

Root finding follows the rational-interpolation scheme of Bunch, Nielsen and
Sorensen (1978) in R.-C. Li's "middle way" form (1993): both pole sums are
modelled by a constant plus one simple pole fitted to value and slope, and
the resulting quadratic is solved for the step.  A bisection safeguard keeps
every iterate inside a bracket on which the secular function changes sign.
``method="bisect"`` runs pure bisection to the last representable bit.
"""

import numpy as np

EPS = np.finfo(np.float64).eps


def _chunks(n, size):
    for a in range(0, n, size):
        yield a, min(n, a + size)


def choose_origins(D, z, rho):
    """Origin index o_j (nearest pole) and half-gap bracket for every root.

    For j < K-1 the root lies in (D_j, D_{j+1}); it is left of the midpoint
    iff f(midpoint) > 0 (f increases on the interval).  Then o_j = j and the
    offset tau lies in (0, h]; otherwise o_j = j+1 and tau in [-h, 0), with
    h = (D_{j+1} - D_j) / 2.  The last root has o = K-1, tau in
    (0, rho ||z||^2].
    """
    K = D.shape[0]
    z2 = z * z
    org = np.empty(K, dtype=np.int64)
    lo = np.empty(K)
    hi = np.empty(K)
    org[K - 1] = K - 1
    lo[K - 1] = 0.0
    # rho ||z||^2 bounds the last root; widened by a few ulps so that a root
    # sitting exactly on the bound stays strictly inside the bracket.
    hi[K - 1] = rho * float(z2.sum()) * (1.0 + 8.0 * EPS)
    if K > 1:
        h = 0.5 * (D[1:] - D[:-1])
        for a, b in _chunks(K - 1, 256):
            j = np.arange(a, b)
            delta = D[None, :] - D[j][:, None] - h[j][:, None]
            fmid = 1.0 + rho * (z2[None, :] / delta).sum(axis=1)
            left = fmid > 0.0
            org[j] = np.where(left, j, j + 1)
            lo[j] = np.where(left, 0.0, -h[j])
            hi[j] = np.where(left, h[j], 0.0)
    return org, lo, hi


def secular_roots(D, z, rho, method="interp", max_iter=200):
    """Roots of the secular function as (org, tau); lam_j = D[org_j] + tau_j.

    D strictly increasing, all z_i != 0, rho > 0.
    """
    D = np.asarray(D, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    K = D.shape[0]
    z2 = z * z
    org, lo, hi = choose_origins(D, z, rho)
    tau = np.empty(K)
    for a, b in _chunks(K, 256):
        tau[a:b] = _solve_chunk(D, z2, rho, np.arange(a, b), org[a:b],
                                lo[a:b].copy(), hi[a:b].copy(), method,
                                max_iter)
    return org, tau


def _solve_chunk(D, z2, rho, j, org, lo, hi, method, max_iter):
    K = D.shape[0]
    J = j.shape[0]
    idx = np.arange(K)
    left_mask = idx[None, :] <= j[:, None]          # poles with i <= j
    delta = D[None, :] - D[org][:, None]
    dj = delta[np.arange(J), j]                      # delta of the left pole
    last = j == K - 1
    dj1 = np.where(last, 0.0, delta[np.arange(J), np.minimum(j + 1, K - 1)])
    tau = 0.5 * (lo + hi)
    done = np.zeros(J, dtype=bool)
    best = tau.copy()
    for _ in range(max_iter):
        t = delta - tau[:, None]
        terms = z2[None, :] / t
        g = 1.0 / rho + terms.sum(axis=1)
        abssum = 1.0 / rho + np.abs(terms).sum(axis=1)
        # Shrink the bracket: g increases in tau.
        pos = g > 0.0
        hi = np.where(~done & pos, tau, hi)
        lo = np.where(~done & ~pos, tau, lo)
        best = np.where(done, best, tau)
        if method == "bisect":
            mid = 0.5 * (lo + hi)
            conv = (mid <= lo) | (mid >= hi) | (g == 0.0)
            done |= conv
            if done.all():
                break
            tau = np.where(done, tau, mid)
            continue
        conv = np.abs(g) <= 8.0 * EPS * abssum
        width = hi - lo
        conv |= width <= 4.0 * EPS * np.maximum(np.abs(lo), np.abs(hi))
        done |= conv
        if done.all():
            break
        # Middle-way model of psi (left poles) and phi (right poles).
        dterms = terms / t
        psi = np.where(left_mask, terms, 0.0).sum(axis=1)
        dpsi = np.where(left_mask, dterms, 0.0).sum(axis=1)
        phi = np.where(left_mask, 0.0, terms).sum(axis=1)
        dphi = np.where(left_mask, 0.0, dterms).sum(axis=1)
        d1 = dj - tau                                # < 0
        d2 = dj1 - tau                               # > 0 (unused when last)
        s1 = dpsi * d1 * d1
        s2 = np.where(last, 0.0, dphi * d2 * d2)
        c = 1.0 / rho + (psi - dpsi * d1) + np.where(last, 0.0, phi - dphi * d2)
        with np.errstate(all="ignore"):
            # last root: c + s1/(d1 - eta) = 0
            eta_last = d1 + s1 / c
            # interior: c eta^2 - B eta + C = 0, one root in (d1, d2)
            B = c * (d1 + d2) + s1 + s2
            C = c * d1 * d2 + s1 * d2 + s2 * d1
            disc = np.maximum(B * B - 4.0 * c * C, 0.0)
            q = 0.5 * (B + np.copysign(np.sqrt(disc), B))
            r1 = q / c
            r2 = C / q
            # the model root inside the current bracket (the other root of the
            # quadratic can also round into (d1, d2) when the root hugs a pole)
            in2 = (r2 > lo - tau) & (r2 < hi - tau)
            eta_int = np.where(in2, r2, r1)
            eta = np.where(last, eta_last, eta_int)
            new = tau + eta
        ok = np.isfinite(new) & (new > lo) & (new < hi)
        new = np.where(ok, new, 0.5 * (lo + hi))
        tau = np.where(done, tau, new)
    else:
        if not done.all():
            raise RuntimeError("secular solver did not converge")
    return best


def secular_value(D, z, rho, org, tau):
    """f at every root, evaluated in the stable (origin, offset) form."""
    out = np.empty(D.shape[0])
    for a, b in _chunks(D.shape[0], 256):
        t = (D[None, :] - D[org[a:b]][:, None]) - tau[a:b][:, None]
        out[a:b] = 1.0 + rho * (z * z / t).sum(axis=1)
    return out


def lam_minus_pole(D, org, tau, rows=None, cols=None):
    """Matrix of lam_j - D_i = (D_{o_j} - D_i) + tau_j (Remark 3)."""
    rows = np.arange(D.shape[0]) if rows is None else rows
    cols = np.arange(org.shape[0]) if cols is None else cols
    return (D[org[cols]][None, :] - D[rows][:, None]) + tau[cols][None, :]


def loewner_z(D, org, tau, z, rho):
    """Gu-Eisenstat recomputation of z from the computed roots.

    zhat_i^2 = (lam_K - D_i)/rho * prod_{j<i} (lam_j - D_i)/(D_j - D_i)
                               * prod_{i<=j<K} (lam_j - D_i)/(D_{j+1} - D_i)
    (0-based j < K-1 in the last product); every factor is positive by
    interlacing.  The sign is taken from z.
    """
    K = D.shape[0]
    zhat = np.empty(K)
    for a, b in _chunks(K, 256):
        i = np.arange(a, b)
        lmd = lam_minus_pole(D, org, tau, rows=i)          # (rows, K): lam_j - D_i
        jj = np.arange(K - 1)
        den_lo = D[None, jj] - D[i][:, None]               # D_j - D_i
        den_hi = D[None, jj + 1] - D[i][:, None]           # D_{j+1} - D_i
        use_lo = jj[None, :] < i[:, None]
        den = np.where(use_lo, den_lo, den_hi)
        ratio = lmd[:, :K - 1] / den
        prod = lmd[:, K - 1] / rho
        prod = prod * np.prod(ratio, axis=1)
        zhat[a:b] = np.sqrt(prod)
    return np.copysign(zhat, z)


def column_scale(D, org, tau, zhat):
    """s_j = (sum_i zhat_i^2 / (D_i - lam_j)^2)^(-1/2) (eq. Q_Cauchy)."""
    K = D.shape[0]
    s = np.empty(K)
    for a, b in _chunks(K, 256):
        cols = np.arange(a, b)
        den = -lam_minus_pole(D, org, tau, cols=cols)       # D_i - lam_j
        s[a:b] = 1.0 / np.sqrt(((zhat[:, None] / den) ** 2).sum(axis=0))
    return s


def cauchy_matrix(D, org, tau, zhat, s, rows=None, cols=None):
    """U_ij = zhat_i s_j / ((D_i - D_{o_j}) - tau_j) (eq. Q_Cauchy, Remark 3).

    With ``org is None`` the generators are general: U_ij = zhat_i s_j /
    (D_i - tau_j), i.e. tau holds the column nodes directly.
    """
    K = D.shape[0]
    rows = np.arange(K) if rows is None else rows
    cols = np.arange(tau.shape[0]) if cols is None else cols
    if org is None:
        den = D[rows][:, None] - tau[cols][None, :]
    else:
        den = (D[rows][:, None] - D[org[cols]][None, :]) - tau[cols][None, :]
    return zhat[rows][:, None] * s[cols][None, :] / den


def solve_rank_one(D, z, rho, method="interp"):
    """(org, tau, zhat, s) for D + rho z z^T: the merge's generators."""
    org, tau = secular_roots(D, z, rho, method=method)
    zhat = loewner_z(D, org, tau, z, rho)
    s = column_scale(D, org, tau, zhat)
    return org, tau, zhat, s
