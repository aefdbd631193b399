"""GPU parity of the generated-tile merge product C = Qnd U (dc_merge_update).

The oracle supplies the generators (its secular solver, Loewner weights and
column scales) and the reference product numpy(Qnd) @ U.  Bound: each entry
is a K-term FP64 dot product, so |C - C_ref| <= 4 K eps (|Qnd| |U|)_ij.
"""
import numpy as np
import pytest

from oracle import secular
from paper_2008_01990_amd import workloads as W
from tests.gpu_util import announce, cuda, host

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


def _run(lib, Qnd, D, org, tau, zhat, s, **kw):
    import torch
    m, K = Qnd.shape
    C = lib.merge_update(cuda(Qnd.T), m, K, cuda(D),
                         None if org is None else cuda(org, torch.int32),
                         cuda(tau), cuda(zhat), cuda(s), **kw)
    return host(C).T


def _bound(Qnd, U):
    return 4 * U.shape[0] * EPS * (np.abs(Qnd) @ np.abs(U)) + 1e-300


# (4096, 4096): 32 x 32 tiles of 128 x 128, more than 8 groups of 64 tiles,
# so the tile order within the task is the transposed (spread) one.
@pytest.mark.parametrize("m,K,seed", [(517, 300, 0), (256, 128, 1), (1, 1, 2), (33, 7, 3),
                                      (1000, 515, 4), (4096, 4096, 5), (4100, 3001, 6)])
def test_plain_merge_update_matches_oracle(lib, m, K, seed):
    announce(f"merge_update m={m} K={K} seed={seed}")
    D, z, rho = W.random_secular(K, seed=seed)
    org, tau, zhat, s = secular.solve_rank_one(D, z, rho)
    Qnd = W.random_matrix(m, K, seed=seed + 10)
    U = secular.cauchy_matrix(D, org, tau, zhat, s)
    ref = Qnd @ U
    got = _run(lib, Qnd, D, org, tau, zhat, s)
    assert np.all(np.abs(got - ref) <= _bound(Qnd, U))


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_tile_variants_agree(lib, variant):
    m, K = 300, 260
    announce(f"merge_update variant={variant}")
    D, z, rho = W.random_secular(K, seed=7)
    org, tau, zhat, s = secular.solve_rank_one(D, z, rho)
    Qnd = W.random_matrix(m, K, seed=8)
    U = secular.cauchy_matrix(D, org, tau, zhat, s)
    got = _run(lib, Qnd, D, org, tau, zhat, s, variant=variant)
    assert np.all(np.abs(got - Qnd @ U) <= _bound(Qnd, U))


def test_general_cauchy_generators(lib):
    # Examples 0/1: U_ij = u_i v_j / (d_i - w_j) with org = NULL.
    n = 384
    announce("merge_update general cauchy n=384")
    u, v, d, w = W.example_cauchy(n, seed=2)
    A = W.random_matrix(200, n, seed=3)
    B = secular.cauchy_matrix(d, None, w, u, v)
    got = _run(lib, A, d, None, w, u, v)
    assert np.all(np.abs(got - A @ B) <= _bound(A, B))
