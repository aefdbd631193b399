"""GPU parity of the secular solver, Loewner weights and column scales.

Roots are compared on the offset scale: two correct solvers may differ in
the last bits of tau (several last-bit answers are all correct), within what
the shared stopping rule leaves open: twice 8 eps sum|terms| / g'(tau) per
root.  Loewner weights and scales are smooth
functions of the roots and agree to ~1e-13 relative.
"""
import numpy as np
import pytest
import torch

from oracle import secular
from paper_2008_01990_amd import workloads as W
from tests.gpu_util import announce, cuda, host

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


# K = 3000 and 4097: several 1024-pole chunks per sweep (and a ragged last one)
@pytest.mark.parametrize("K,seed,cluster", [(1, 0, False), (2, 1, False), (63, 2, False),
                                            (700, 3, False), (300, 4, True), (200, 5, True),
                                            (256, 6, False), (3000, 7, False),
                                            (4097, 8, True)])
def test_secular_matches_oracle(lib, K, seed, cluster):
    announce(f"secular K={K} seed={seed} cluster={cluster}")
    D, z, rho = W.random_secular(K, seed=seed, cluster=cluster)
    o_org, o_tau, o_zhat, o_s = secular.solve_rank_one(D, z, rho)
    g_org, g_tau, g_zhat, g_s = [host(t) for t in lib.secular(D, z, rho)]
    g_org = g_org.astype(np.int64)
    # same root, possibly different frame: (D[og] - D[oo]) + (tg - to)
    diff = (D[g_org] - D[o_org]) + (g_tau - o_tau)
    # Each solver stops at |g(tau)| <= 8 eps sum_i |z_i^2 / (delta_i - tau)|
    # (or a 4-ulp bracket), so each root is off by at most that over the
    # slope g'(tau) = sum_i z_i^2 / (delta_i - tau)^2: two correct answers may
    # differ by twice it.  (Relative to tau the bound reaches ~300 ulps on
    # some roots of K = 3000, where the oracle's own interpolating and
    # bisecting solvers differ by up to 105 ulps of tau.)
    cond = np.empty(K)
    z2 = z * z
    for j in range(K):
        t = (D - D[o_org[j]]) - o_tau[j]
        cond[j] = 8 * EPS * (1 / rho + np.abs(z2 / t).sum()) / (z2 / t ** 2).sum()
    bound = 2 * cond + 4 * EPS * (np.abs(o_tau) + np.abs(D[g_org] - D[o_org]))
    assert np.all(np.abs(diff) <= bound)
    lam = D[g_org] + g_tau
    assert np.all(lam[:-1] > D[:-1]) and np.all(lam[:-1] < D[1:])
    assert np.allclose(g_zhat, o_zhat, rtol=1e-12, atol=0)
    assert np.allclose(g_s, o_s, rtol=1e-12, atol=0)
    U = secular.cauchy_matrix(D, g_org, g_tau, g_zhat, g_s)
    assert np.abs(U.T @ U - np.eye(K)).max() <= 1e-13


def test_secular_max_iter_one_sets_status(lib):
    # A one-iteration cap: the kernel stops the unconverged roots and the
    # status word holds the first one's 1-based index.
    K = 500
    D, z, rho = W.random_secular(K, seed=11)
    announce("secular max_iter=1 status")
    Dd, zd = cuda(D), cuda(z)
    org = torch.empty(K, dtype=torch.int32, device="cuda")
    tau, zhat, s = (torch.empty(K, dtype=torch.float64, device="cuda") for _ in range(3))
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    L = lib.load()
    rc = L.dc_secular(K, lib._ptr(Dd), lib._ptr(zd), float(rho), lib._ptr(org), lib._ptr(tau),
                      lib._ptr(zhat), lib._ptr(s), lib._ptr(info), 1, lib._stream())
    assert rc == 0
    st = int(info.item())
    assert 1 <= st <= K, st
    with pytest.raises(lib.DcError):
        lib.secular(D, z, rho, max_iter=1)
