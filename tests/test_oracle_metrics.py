"""Pins for the oracle's accuracy measures and its secular-function helper.

Each measure is checked on inputs whose value is known in closed form, not by
re-evaluating its own formula.
"""
import numpy as np
import pytest

from oracle import metrics, secular
from paper_2008_01990_amd import workloads as W


def _toeplitz_exact(n):
    k = np.arange(1, n + 1)
    lam = 2.0 - 2.0 * np.cos(k * np.pi / (n + 1))
    i = np.arange(1, n + 1)[:, None]
    Q = np.sqrt(2.0 / (n + 1)) * np.sin(i * k[None, :] * np.pi / (n + 1))
    return lam, Q


@pytest.mark.parametrize("n", [5, 40, 200])
def test_paper_residual_identity_basis(n):
    # Q = I, lam = d on the 1-2-1 matrix: A - Q Lambda Q^T is the
    # off-diagonal part, whose interior columns have norm sqrt(2); ||A||_2 is
    # the largest eigenvalue 2 + 2 cos(pi / (n + 1)).
    d, e = W.toeplitz(n)
    got = metrics.paper_residual(d, e, d, np.eye(n))
    assert got == pytest.approx(np.sqrt(2.0) / (2.0 + 2.0 * np.cos(np.pi / (n + 1))),
                                rel=1e-14)


def test_paper_residual_exact_and_one_shifted_eigenvalue():
    n = 64
    d, e = W.toeplitz(n)
    lam, Q = _toeplitz_exact(n)
    assert metrics.paper_residual(d, e, lam, Q) <= 1e-14
    # lam_j off by delta: the residual is delta q_j q_j^T, whose largest
    # column norm is delta max_i |q_ij|.
    j, delta = 17, 1e-6
    lam2 = lam.copy()
    lam2[j] += delta
    want = delta * np.abs(Q[:, j]).max() / (2.0 + 2.0 * np.cos(np.pi / (n + 1)))
    assert metrics.paper_residual(d, e, lam2, Q) == pytest.approx(want, rel=1e-8)


def test_paper_orthogonality_uses_rows():
    # Q = I + a (E_01 + E_02): Q Q^T - I has (0, 0) entry 2 a^2, while
    # Q^T Q - I peaks at a^2 off the diagonal; for a = 2 the two measures are
    # 8 and 4.
    Q = np.eye(3)
    Q[0, 1] = Q[0, 2] = 2.0
    assert metrics.paper_orthogonality(Q) == 8.0
    assert metrics.orthogonality(Q) == 4.0
    lam, S = _toeplitz_exact(50)
    assert metrics.paper_orthogonality(S) <= 1e-14


@pytest.mark.parametrize("K,seed", [(6, 0), (25, 1)])
def test_secular_value_matches_determinant_ratio(K, seed):
    # Matrix determinant lemma: det(D + rho z z^T - lam I) / det(D - lam I)
    # = 1 + rho sum z_i^2 / (D_i - lam), for lam given as (origin, offset)
    # anywhere off the poles.
    D, z, rho = W.random_secular(K, seed=seed)
    M = np.diag(D) + rho * np.outer(z, z)
    rng = np.random.default_rng(seed + 10)
    org = rng.integers(0, K, K)          # one evaluation point per pole slot
    gaps = np.diff(np.concatenate([D, [D[-1] + 1.0]]))
    tau = rng.uniform(0.1, 0.9, K) * gaps[org]
    f = secular.secular_value(D, z, rho, org, tau)
    for a in range(K):
        lam = D[org[a]] + tau[a]
        s1, l1 = np.linalg.slogdet(M - lam * np.eye(K))
        s2, l2 = np.linalg.slogdet(np.diag(D) - lam * np.eye(K))
        assert f[a] == pytest.approx(s1 * s2 * np.exp(l1 - l2), rel=1e-9)


def test_secular_value_vanishes_at_dense_eigenvalues():
    # The eigenvalues of the dense rank-one problem (LAPACK), written as
    # (nearest pole, offset), are zeros of f up to rounding of the sum.
    K = 40
    D, z, rho = W.random_secular(K, seed=3)
    lam = np.linalg.eigvalsh(np.diag(D) + rho * np.outer(z, z))
    org = np.argmin(np.abs(lam[:, None] - D[None, :]), axis=1)
    tau = lam - D[org]
    f = secular.secular_value(D, z, rho, org, tau)
    absf = np.array([1 + rho * np.abs(z * z / ((D - D[o]) - t)).sum() for o, t in zip(org, tau)])
    assert np.all(np.abs(f) <= 1e-9 * absf)
