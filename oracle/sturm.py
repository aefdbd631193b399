"""Sturm-sequence bisection for tridiagonal eigenvalues.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Independent of divide and conquer: the number of eigenvalues of T(d, e)
below x equals the number of negative pivots of the LDL^T factorisation of
T - x I (Sylvester's law of inertia; Golub & Van Loan section 8.4).  Each
eigenvalue is then bracketed by Gershgorin bounds and bisected to adjacent
doubles.
"""

import numpy as np

_TINY = np.finfo(np.float64).tiny


def count_below(d, e, x):
    """Number of eigenvalues of T(d, e) strictly less than x."""
    cnt = 0
    q = d[0] - x
    if q < 0.0:
        cnt += 1
    for i in range(1, d.shape[0]):
        if q == 0.0:
            q = _TINY
        q = (d[i] - x) - e[i - 1] * e[i - 1] / q
        if q < 0.0:
            cnt += 1
    return cnt


def eigvals(d, e):
    """All eigenvalues, ascending, each bisected to the last bit."""
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    n = d.shape[0]
    r = np.zeros(n)
    if n > 1:
        r[:-1] += np.abs(e)
        r[1:] += np.abs(e)
    glo = float((d - r).min())
    ghi = float((d + r).max())
    span = max(abs(glo), abs(ghi), 1.0)
    glo -= 4 * np.finfo(float).eps * span
    ghi += 4 * np.finfo(float).eps * span
    out = np.empty(n)
    for k in range(n):
        lo, hi = glo, ghi            # count_below(lo) <= k < count_below(hi)
        while True:
            mid = 0.5 * (lo + hi)
            if mid <= lo or mid >= hi:
                break
            if count_below(d, e, mid) > k:
                hi = mid
            else:
                lo = mid
        out[k] = hi if abs(hi - lo) == 0 else 0.5 * (lo + hi)
    return out
