"""Pins for the oracle's leaf QR (Algorithm 1's small-block solver)."""
import numpy as np
import pytest

from oracle import leaf, metrics, sturm
from paper_2008_01990_amd import workloads as W


@pytest.mark.parametrize("n", [1, 2, 3, 7, 32, 64])
def test_leaf_matches_sturm_bisection(n):
    rng = np.random.default_rng(n)
    d, e = W.random_tridiag(n, rng)
    lam, Q = leaf.tridiag_qr(d, e)
    ref = sturm.eigvals(d, e)
    tn = max(np.abs(ref).max(), 1.0)
    assert np.abs(lam - ref).max() <= 1e-14 * tn
    assert metrics.orthogonality(Q) <= 1e-14
    assert metrics.residual(d, e, lam, Q) <= 1e-15


def test_leaf_two_by_two_closed_form():
    a, b, c = 0.3, -1.7, 0.9
    lam, Q = leaf.tridiag_qr([a, c], [b])
    mean, rad = 0.5 * (a + c), np.hypot(0.5 * (a - c), b)
    assert np.allclose(lam, [mean - rad, mean + rad], atol=1e-15, rtol=0)
    T = np.array([[a, b], [b, c]])
    assert np.abs(T @ Q - Q * lam).max() < 1e-15


def test_leaf_diagonal_and_zero_offdiagonal():
    d = np.array([3.0, -1.0, 2.0, 2.0, 0.5])
    lam, Q = leaf.tridiag_qr(d, np.zeros(4))
    assert np.array_equal(lam, np.sort(d))
    assert metrics.orthogonality(Q) == 0.0


def test_leaf_toeplitz_closed_form():
    n = 48
    d, e = W.toeplitz(n)
    lam, Q = leaf.tridiag_qr(d, e)
    k = np.arange(1, n + 1)
    ref = 2.0 - 2.0 * np.cos(k * np.pi / (n + 1))
    assert np.abs(lam - ref).max() <= 8 * np.finfo(float).eps * 4.0
    i = np.arange(1, n + 1)[:, None]
    S = np.sqrt(2.0 / (n + 1)) * np.sin(i * k[None, :] * np.pi / (n + 1))
    # eigenvectors up to sign
    assert np.abs(np.abs((S * Q).sum(axis=0)) - 1.0).max() <= 1e-12


def test_leaf_zero_diagonal_converges():
    # Clement-type blocks have d = 0: a relative deflation test would stall.
    d, e = W.clement(33)
    lam, Q = leaf.tridiag_qr(d, e)
    assert np.allclose(lam, np.arange(-32.0, 33.0, 2.0), atol=1e-13, rtol=0)
