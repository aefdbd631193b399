"""Element-wise eigenvector comparison shared by the GPU parity tests.

An eigenvector is determined only up to sign and, individually, only to
about eps ||T|| / gap_j, where gap_j is the distance from lambda_j to the
nearest other eigenvalue.  So the columns are sign-aligned and compared entry
by entry:

    max_i |q_ij - s_j qo_ij| <= C eps ||T|| / gap_j + FLOOR,   s_j = sign(q_j . qo_j).

The error is linear in the perturbation of the vector (a dot-product test
1 - |q . qo| = ||q - qo||^2 / 2 is quadratic and lets a column off by 1e-6
pass at a 1e-12 bar).  C = 100: an independent solver (LAPACK's MRRR via
SciPy) against the oracle reaches at most 4.4 eps ||T|| / gap_j on the
families used here, so the bar leaves a margin of about 20.  Columns whose
eigenvalue has a (numerically) equal neighbour have no individual vector to
compare; their bound exceeds 1 and they are skipped, the invariant subspace
being covered by the residual and orthogonality bars.
"""
import numpy as np

EPS = np.finfo(float).eps
C_VEC = 100.0
FLOOR = 100.0 * EPS


def gaps(lam):
    lam = np.asarray(lam, dtype=np.float64)
    n = lam.shape[0]
    gap = np.full(n, np.inf)
    if n > 1:
        g = np.diff(lam)
        gap[:-1] = np.minimum(gap[:-1], g)
        gap[1:] = np.minimum(gap[1:], g)
    return gap


def eigvec_bound(lam_ref, tn=None):
    """Per-column element-wise bound C eps ||T|| / gap_j + FLOOR."""
    tn = float(np.abs(lam_ref).max()) if tn is None else tn
    with np.errstate(divide="ignore"):
        return C_VEC * EPS * max(tn, 1e-300) / gaps(lam_ref) + FLOOR


def assert_eigvecs_match(Q, Qo, lam_ref, tn=None, cols=None):
    """Q and Qo (n x n or n x len(cols)) column j against column j, up to sign.

    lam_ref: the reference eigenvalues (all n), used for the gaps; cols
    selects the columns of the full spectrum that Q and Qo hold (default all).
    """
    Q = np.asarray(Q)
    Qo = np.asarray(Qo)
    bound = eigvec_bound(lam_ref, tn)
    if cols is not None:
        bound = bound[np.asarray(cols)]
    s = np.sign((Q * Qo).sum(axis=0))
    s[s == 0] = 1.0
    err = np.abs(Q - Qo * s[None, :]).max(axis=0) if Q.shape[0] else np.zeros(Q.shape[1])
    check = bound < 1.0
    bad = np.flatnonzero(check & (err > bound))
    assert bad.size == 0, (
        f"{bad.size} eigenvector columns off: worst column {bad[np.argmax(err[bad] / bound[bad])]}"
        f" err {err[bad].max():.3e} vs bound {bound[bad][np.argmax(err[bad])]:.3e}")
    return err, bound


def residual_eig_bound(d, e, lam, Q):
    """Per column ||T q_j - lam_j q_j|| / ||q_j||: for symmetric T, lam_j is
    within this distance of an eigenvalue of T (the residual bound), whether
    or not q_j is exactly orthogonal to the other columns."""
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    Y = d[:, None] * Q
    if d.shape[0] > 1:
        Y[:-1] += e[:, None] * Q[1:]
        Y[1:] += e[:, None] * Q[:-1]
    R = Y - Q * np.asarray(lam)[None, :]
    return np.linalg.norm(R, axis=0) / np.linalg.norm(Q, axis=0)


def assert_lowrank_eigvals(d, e, lam, Q, lam_ref, floor=1e-13):
    """Low-rank path: |lam_j - lam_ref_j| <= residual bound of column j +
    floor ||T||.  The low-rank merge returns approximate eigenpairs (its U is
    within tol of the exact one entry by entry), so the eigenvalues are held
    to what their own residuals guarantee, plus the plain path's bar."""
    tn = float(np.abs(lam_ref).max())
    bound = residual_eig_bound(d, e, lam, Q) + floor * tn
    err = np.abs(np.asarray(lam) - np.asarray(lam_ref))
    assert np.all(err <= bound), (err.max() / tn, int(np.argmax(err / bound)))
    return err, bound
