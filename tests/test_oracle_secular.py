"""Pins for the oracle's secular solver, Loewner z and Cauchy eigenvectors.

Pins: closed forms for K = 1 and K = 2, interlacing, agreement with pure
bisection to the last bit, the dense eigenproblem of D + rho z z^T through
numpy's symmetric eigensolver (library routine), and orthogonality of U.
"""
import numpy as np
import pytest

from oracle import secular as S
from paper_2008_01990_amd import workloads as W


def _lam(D, org, tau):
    return D[org] + tau


def test_single_pole_closed_form():
    D, z, rho = np.array([0.7]), np.array([-0.6]), 1.3
    org, tau = S.secular_roots(D, z, rho)
    assert org[0] == 0
    assert abs(tau[0] - rho * 0.36) <= 1e-16
    zhat = S.loewner_z(D, org, tau, z, rho)
    assert abs(zhat[0] - z[0]) <= 1e-16
    s = S.column_scale(D, org, tau, zhat)
    U = S.cauchy_matrix(D, org, tau, zhat, s)
    assert abs(abs(U[0, 0]) - 1.0) <= 1e-15


def test_two_poles_closed_form():
    D = np.array([-0.5, 1.25])
    z = np.array([0.6, 0.8])
    rho = 0.9
    M = np.diag(D) + rho * np.outer(z, z)
    tr, det = np.trace(M), np.linalg.det(M)
    disc = np.sqrt(tr * tr - 4 * det)
    ref = np.array([(tr - disc) / 2, (tr + disc) / 2])
    org, tau = S.secular_roots(D, z, rho)
    assert np.abs(_lam(D, org, tau) - ref).max() <= 4e-16


@pytest.mark.parametrize("seed,K,cluster", [(0, 50, False), (1, 200, False),
                                            (2, 300, True)])
def test_roots_interlace_and_match_bisection(seed, K, cluster):
    D, z, rho = W.random_secular(K, seed=seed, cluster=cluster)
    org, tau = S.secular_roots(D, z, rho)
    lam = _lam(D, org, tau)
    assert np.all(lam[:-1] > D[:-1]) and np.all(lam[:-1] < D[1:])
    assert lam[-1] > D[-1] and lam[-1] <= D[-1] + rho * (z * z).sum() * (1 + 1e-15)
    ob, tb = S.secular_roots(D, z, rho, method="bisect")
    assert np.array_equal(ob, org)
    # both are within a few ulps of the root measured on the offset scale
    scale = np.maximum(np.abs(tau), np.abs(tb))
    assert np.all(np.abs(tau - tb) <= 64 * np.finfo(float).eps * scale)


def test_roots_match_dense_eigensolver():
    D, z, rho = W.random_secular(120, seed=5)
    org, tau = S.secular_roots(D, z, rho)
    ref = np.linalg.eigvalsh(np.diag(D) + rho * np.outer(z, z))
    tn = np.abs(ref).max()
    assert np.abs(_lam(D, org, tau) - ref).max() <= 1e-14 * tn


def test_origin_is_nearest_pole():
    D, z, rho = W.random_secular(80, seed=6)
    org, tau = S.secular_roots(D, z, rho)
    lam = _lam(D, org, tau)
    j = np.arange(79)
    near = np.where(lam[j] - D[j] <= D[j + 1] - lam[j], j, j + 1)
    assert np.array_equal(org[:-1], near)


@pytest.mark.parametrize("cluster", [False, True])
def test_loewner_reproduces_z_and_u_is_orthogonal(cluster):
    D, z, rho = W.random_secular(256, seed=7, cluster=cluster)
    org, tau, zhat, s = S.solve_rank_one(D, z, rho)
    assert np.all(np.sign(zhat) == np.sign(z))
    assert np.abs(zhat - z).max() <= 1e-12
    U = S.cauchy_matrix(D, org, tau, zhat, s)
    assert np.abs(U.T @ U - np.eye(256)).max() <= 1e-13
    # columns are eigenvectors of the rank-one update
    M = np.diag(D) + rho * np.outer(z, z)
    lam = _lam(D, org, tau)
    assert np.abs(M @ U - U * lam).max() <= 1e-13 * np.abs(lam).max()


def test_secular_value_small_at_roots():
    D, z, rho = W.random_secular(400, seed=8)
    org, tau = S.secular_roots(D, z, rho)
    f = S.secular_value(D, z, rho, org, tau)
    absf = np.array([1 + rho * np.abs(z * z / ((D - D[o]) - t)).sum()
                     for o, t in zip(org, tau)])
    assert np.all(np.abs(f) <= 64 * np.finfo(float).eps * absf)


def test_general_cauchy_generators():
    u, v, d, w = W.example_cauchy(64, seed=1)
    U = S.cauchy_matrix(d, None, w, u, v)
    assert np.allclose(U, u[:, None] * v[None, :] / (d[:, None] - w[None, :]),
                       rtol=0, atol=0)
