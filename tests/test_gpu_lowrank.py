"""GPU parity of the structured low-rank merge (SRRSC compression + products).

The low-rank path is an approximation defined by the oracle: every
off-diagonal b x b block of U replaced by its complete-pivoting SRRSC form at
tolerance tol (oracle.srrsc.lowrank_cauchy).  Both sides choose pivots from
rounded values, so near-ties may pick different pivots; each side's U is
within tol of the exact U entry by entry, hence
  |C_gpu - Qnd U_exact| <= tol * sum_k |Qnd_ik| + rounding,
and the ranks agree up to such ties.
"""
import numpy as np
import pytest
import torch

from oracle import dc, metrics, secular, srrsc
from paper_2008_01990_amd import workloads as W
from tests.gpu_util import announce, cuda, host

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


def _gens(K, seed):
    D, z, rho = W.random_secular(K, seed=seed)
    return D, secular.solve_rank_one(D, z, rho)


@pytest.mark.parametrize("m,K,b,tol,seed", [(700, 1000, 256, 1e-10, 0),
                                           (333, 777, 128, 1e-8, 1)])
def test_lowrank_merge_update_within_tolerance(lib, m, K, b, tol, seed):
    announce(f"lowrank merge_update m={m} K={K} b={b} tol={tol}")
    D, (org, tau, zhat, s) = _gens(K, seed)
    Qnd = W.random_matrix(m, K, seed=seed + 5)
    U = secular.cauchy_matrix(D, org, tau, zhat, s)
    C = host(lib.merge_update(cuda(Qnd.T), m, K, cuda(D), cuda(org, torch.int32), cuda(tau),
                              cuda(zhat), cuda(s), lr_tol=tol, lr_block=b)).T
    exact = Qnd @ U
    bound = tol * np.abs(Qnd).sum(axis=1)[:, None] * 1.01 + 8 * K * EPS * (np.abs(Qnd) @ np.abs(U))
    assert np.all(np.abs(C - exact) <= bound)
    # against the oracle's own approximation
    Ulr, ranks_o = srrsc.lowrank_cauchy(D, org, tau, zhat, s, tol, b)
    assert np.all(np.abs(C - Qnd @ Ulr) <= 2 * bound)
    ranks_g = lib.merge_lowrank_ranks(cuda(D), cuda(org, torch.int32), cuda(tau), cuda(zhat),
                                      cuda(s), tol, b)
    off = ranks_o >= 0
    assert np.array_equal(ranks_g < 0, ranks_o < 0)
    assert np.abs(ranks_g[off] - ranks_o[off]).max() <= 1
    assert (ranks_g[off] == ranks_o[off]).mean() >= 0.9


def test_lowrank_dense_fallback(lib):
    # b = 16 caps the rank at 8; at tol 1e-15 most blocks keep dense.
    K, m, b = 96, 50, 16
    announce("lowrank dense fallback")
    D, (org, tau, zhat, s) = _gens(K, 3)
    Qnd = W.random_matrix(m, K, seed=4)
    U = secular.cauchy_matrix(D, org, tau, zhat, s)
    ranks = lib.merge_lowrank_ranks(cuda(D), cuda(org, torch.int32), cuda(tau), cuda(zhat),
                                    cuda(s), 1e-15, b)
    assert (ranks == -2).any()
    C = host(lib.merge_update(cuda(Qnd.T), m, K, cuda(D), cuda(org, torch.int32), cuda(tau),
                              cuda(zhat), cuda(s), lr_tol=1e-15, lr_block=b)).T
    bound = 1e-15 * np.abs(Qnd).sum(axis=1)[:, None] * 1.01 + 8 * K * EPS * (np.abs(Qnd) @ np.abs(U))
    assert np.all(np.abs(C - Qnd @ U) <= bound)


def test_lowrank_general_cauchy_example1(lib):
    # Example 1's B: d_i = i (b-a)/n, w_j = d_j + (b-a)/(2n), u, v ~ U(0, 1).
    n, b, tol = 1024, 256, 1e-10
    announce("lowrank example1 n=1024")
    u, v, d, w = W.example_cauchy(n, seed=5)
    A = W.random_matrix(300, n, seed=6)
    B = secular.cauchy_matrix(d, None, w, u, v)
    C = host(lib.merge_update(cuda(A.T), 300, n, cuda(d), None, cuda(w), cuda(u), cuda(v),
                              lr_tol=tol, lr_block=b)).T
    bound = tol * np.abs(A).sum(axis=1)[:, None] * 1.01 + 8 * n * EPS * (np.abs(A) @ np.abs(B))
    assert np.all(np.abs(C - A @ B) <= bound)


@pytest.mark.parametrize("family,n", [("toeplitz", 2048), ("clement", 2048)])
def test_lowrank_solver_meets_bounds(lib, family, n):
    announce(f"lowrank stedc {family} n={n}")
    d, e = W.toeplitz(n) if family == "toeplitz" else W.clement(n)
    kw = dict(leaf=64, lr_tol=1e-10, lr_block=256, lr_min_k=512)
    lam, Q = lib.stedc(cuda(d), cuda(e), **kw)
    stats = lib.last_stats()
    assert any(r["path"] == 1 for r in stats)
    lam, Q = host(lam), host(Q)
    if family == "toeplitz":
        k = np.arange(1, n + 1)
        ref = 2 - 2 * np.cos(k * np.pi / (n + 1))
    else:
        ref = np.arange(-(n - 1), n, 2, dtype=float)
    assert metrics.eig_error(lam, ref) <= 1e-13
    assert metrics.orthogonality(Q) <= 1e-9
    assert metrics.residual(d, e, lam, Q) <= 1e-9
    lo, Qo = dc.eigh_tridiagonal(d, e, leaf=64, lr_tol=1e-10, lr_block=256, lr_min_k=512)
    # both sides perturb U by up to tol per entry: eigenvalues move at ~tol scale
    assert np.abs(lam - lo).max() <= 1e-11 * np.abs(lo).max()
