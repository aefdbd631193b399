"""Pins for the oracle's divide and conquer (Algorithm 1 / 3).

Pins: closed-form spectra and eigenvectors (1-2-1 Toeplitz, Clement),
Sturm-sequence bisection, the trace and Frobenius invariants, the exact tear
and rank-one reduction identities (eq. T2 / eq. T3), deflation special cases,
the persymmetric top merge (K = m / 2) and a library cross-check.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dc, metrics, sturm
from paper_2008_01990_amd import workloads as W

EPS = np.finfo(float).eps


def dense(d, e):
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


def test_toeplitz_closed_form_n1024():
    n = 1024
    d, e = W.toeplitz(n)
    log = dc.MergeLog()
    lam, Q = dc.eigh_tridiagonal(d, e, leaf=32, log=log)
    k = np.arange(1, n + 1)
    ref = 2.0 - 2.0 * np.cos(k * np.pi / (n + 1))
    assert metrics.eig_error(lam, ref) <= 1e-14
    assert metrics.orthogonality(Q) <= 1e-13
    assert metrics.residual(d, e, lam, Q) <= 1e-15
    # sine eigenvectors, up to sign; min gap 2.8e-5 fixes them to ~1e-11
    i = np.arange(1, n + 1)[:, None]
    S = math.sqrt(2.0 / (n + 1)) * np.sin(i * k[None, :] * np.pi / (n + 1))
    assert np.abs(np.abs((S * Q).sum(axis=0)) - 1.0).max() <= 1e-10
    # persymmetric halves have equal spectra: the top merge deflates half
    top = log.records[-1]
    assert top["m"] == n and top["K"] == n // 2


def test_clement_closed_form():
    n = 640
    d, e = W.clement(n)
    lam, Q = dc.eigh_tridiagonal(d, e, leaf=64)
    ref = np.arange(-(n - 1), n, 2, dtype=float)
    assert metrics.eig_error(lam, ref) <= 1e-14
    assert metrics.orthogonality(Q) <= 1e-13
    assert metrics.residual(d, e, lam, Q) <= 1e-15


@pytest.mark.parametrize("n,leaf", [(5, 1), (17, 2), (40, 4), (64, 8)])
def test_random_against_sturm(n, leaf):
    rng = np.random.default_rng(100 + n)
    d, e = W.random_tridiag(n, rng)
    lam, Q = dc.eigh_tridiagonal(d, e, leaf=leaf, method="bisect")
    ref = sturm.eigvals(d, e)
    assert metrics.eig_error(lam, ref) <= 1e-14
    assert metrics.orthogonality(Q) <= 1e-14
    assert metrics.residual(d, e, lam, Q) <= 1e-15


def test_invariants_and_library_crosscheck():
    rng = np.random.default_rng(11)
    d, e = W.random_tridiag(333, rng)
    lam, Q = dc.eigh_tridiagonal(d, e, leaf=16)
    assert abs(lam.sum() - d.sum()) <= 1e-12
    assert abs((lam ** 2).sum() - ((d ** 2).sum() + 2 * (e ** 2).sum())) <= 1e-11
    ref = sla.eigh_tridiagonal(d, e, eigvals_only=True)
    assert metrics.eig_error(lam, ref) <= 1e-14
    assert np.all(np.diff(lam) >= 0)


def test_tear_identity_exact():
    rng = np.random.default_rng(12)
    d, e = W.random_tridiag(9, rng)
    for k in range(1, 9):
        d1, e1, d2, e2, rho, sigma = dc.tear(d, e, k)
        w = np.zeros(9)
        w[k - 1] = 1.0
        w[k] = sigma
        T = np.zeros((9, 9))
        T[:k, :k] = dense(d1, e1)
        T[k:, k:] = dense(d2, e2)
        T += rho * np.outer(w, w)
        assert np.array_equal(T, dense(d, e))


def test_rank_one_reduction_identity():
    rng = np.random.default_rng(13)
    d, e = W.random_tridiag(30, rng)
    k = 15
    d1, e1, d2, e2, rho, sigma = dc.tear(d, e, k)
    l1, Q1 = dc.eigh_tridiagonal(d1, e1, leaf=4)
    l2, Q2 = dc.eigh_tridiagonal(d2, e2, leaf=4)
    z = np.concatenate([Q1[-1], sigma * Q2[0]]) / math.sqrt(2.0)
    assert abs(np.linalg.norm(z) - 1.0) <= 1e-15
    B = sla.block_diag(Q1, Q2)
    M = np.diag(np.concatenate([l1, l2])) + 2 * rho * np.outer(z, z)
    assert np.abs(B @ M @ B.T - dense(d, e)).max() <= 1e-14


def test_special_sizes():
    lam, Q = dc.eigh_tridiagonal([3.5], [])
    assert lam.tolist() == [3.5] and Q.tolist() == [[1.0]]
    lam, Q = dc.eigh_tridiagonal([1.0, 1.0], [2.0], leaf=1)
    assert np.allclose(lam, [-1.0, 3.0], atol=1e-15, rtol=0)
    assert metrics.orthogonality(Q) <= 1e-15


def test_zero_coupling_deflates_everything():
    # e == 0 at every split: rho = 0, every merge deflates completely.
    d = np.array([4.0, -2.0, 7.0, 1.0, 1.0, 0.0, -3.0, 5.0])
    log = dc.MergeLog()
    lam, Q = dc.eigh_tridiagonal(d, np.zeros(7), leaf=1, log=log)
    assert np.array_equal(lam, np.sort(d))
    assert all(r["K"] == 0 for r in log.records)
    assert np.array_equal(np.abs(Q).sum(axis=0), np.ones(8))


def test_pair_rotation_deflation():
    # Mirror-image halves have equal spectra after the tear (T2' is T1'
    # reversed), so every pole appears twice and pairs are rotated away.
    blk_d, blk_e = np.array([1.0, 2.0, 3.0, 4.0]), np.array([0.5, 0.5, 0.5])
    d = np.concatenate([blk_d, blk_d[::-1]])
    e = np.concatenate([blk_e, [0.25], blk_e])
    log = dc.MergeLog()
    lam, Q = dc.eigh_tridiagonal(d, e, leaf=4, log=log)
    rec = log.records[-1]
    assert rec["nrot"] >= 1 and rec["K"] < 8
    ref = np.linalg.eigvalsh(dense(d, e))
    assert metrics.eig_error(lam, ref) <= 1e-14
    assert metrics.orthogonality(Q) <= 1e-14
    assert metrics.residual(d, e, lam, Q) <= 1e-15


def test_lowrank_variant_meets_bound():
    n = 2048
    d, e = W.toeplitz(n)
    log = dc.MergeLog()
    lam, Q = dc.eigh_tridiagonal(d, e, leaf=64, lr_tol=1e-10, lr_block=256,
                                 lr_min_k=512, log=log)
    assert any(r["path"] == "lowrank" for r in log.records)
    k = np.arange(1, n + 1)
    assert metrics.eig_error(lam, 2 - 2 * np.cos(k * np.pi / (n + 1))) <= 1e-13
    assert metrics.orthogonality(Q) <= 1e-9
    assert metrics.residual(d, e, lam, Q) <= 1e-9
    for r in log.records:
        if r["path"] == "lowrank":
            rk = r["ranks"][r["ranks"] >= 0]
            assert rk.max() <= 40      # off-diagonal blocks are low rank


def test_hermite_type_against_hermite_roots():
    # d = 0, e_i = sqrt(i): the Jacobi matrix of the probabilists' Hermite
    # polynomials; its eigenvalues are their roots (SciPy, library routine).
    from scipy.special import roots_hermitenorm
    n = 300
    d, e = W.hermite(n)
    lam, Q = dc.eigh_tridiagonal(d, e, leaf=32)
    ref = np.sort(roots_hermitenorm(n)[0])
    assert metrics.eig_error(lam, ref) <= 1e-13
    assert metrics.orthogonality(Q) <= 1e-13
    assert metrics.residual(d, e, lam, Q) <= 1e-15


def test_sht_matrix_definition_and_solve():
    # Example 3's SHT matrix: spot values from its formula and a solve that
    # matches Sturm bisection.
    n = 48
    d, e = W.sht(n)
    m = n
    l0 = m
    assert abs(d[0] - (2 * l0 * (l0 + 1) - 2 * m * m - 1) / ((2 * l0 - 1) * (2 * l0 + 3))) <= 1e-15
    c0 = np.sqrt(1 * 2 * (2 * m + 1) * (2 * m + 2) / ((2 * l0 + 1) * (2 * l0 + 3) ** 2 * (2 * l0 + 5)))
    assert abs(e[0] - c0) <= 1e-15
    lam, Q = dc.eigh_tridiagonal(d, e, leaf=8)
    assert metrics.eig_error(lam, sturm.eigvals(d, e)) <= 1e-14
    assert metrics.orthogonality(Q) <= 1e-14
