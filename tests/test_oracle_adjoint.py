"""Pins for the oracle's dense adjoint: Hellmann-Feynman and finite differences."""
import numpy as np

from oracle import adjoint
from paper_2008_01990_amd import workloads as W


def _eigh(d, e):
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    return np.linalg.eigh(T)


def test_hellmann_feynman_eigenvalue_part():
    rng = np.random.default_rng(0)
    d, e = W.random_tridiag(20, rng)
    lam, Q = _eigh(d, e)
    lb = rng.standard_normal(20)
    db, eb = adjoint.backward(lam, Q, lam_bar=lb)
    assert np.allclose(db, (Q * Q) @ lb, atol=1e-14, rtol=0)
    assert np.allclose(eb, 2 * (Q[:-1] * Q[1:]) @ lb, atol=1e-14, rtol=0)


def _loss(d, e, w, c, u):
    lam, Q = _eigh(d, e)
    return float(w @ lam + c @ (u @ Q) ** 2)


def test_finite_differences_full_loss():
    rng = np.random.default_rng(1)
    n = 14
    d = 2 + 0.3 * rng.standard_normal(n)
    e = -1 + 0.3 * rng.standard_normal(n - 1)
    w, c, u = rng.standard_normal((3, n))
    lam, Q = _eigh(d, e)
    a = u @ Q
    Qb = np.outer(u, 2 * c * a)          # d/dQ of sum c_i (u^T q_i)^2
    db, eb = adjoint.backward(lam, Q, lam_bar=w, Q_bar=Qb)
    h = 1e-6
    for i in range(n):
        dp, dm = d.copy(), d.copy()
        dp[i] += h
        dm[i] -= h
        fd = (_loss(dp, e, w, c, u) - _loss(dm, e, w, c, u)) / (2 * h)
        assert abs(fd - db[i]) <= 1e-6 * max(1.0, abs(fd))
    for i in range(n - 1):
        ep, em = e.copy(), e.copy()
        ep[i] += h
        em[i] -= h
        fd = (_loss(d, ep, w, c, u) - _loss(d, em, w, c, u)) / (2 * h)
        assert abs(fd - eb[i]) <= 1e-6 * max(1.0, abs(fd))
