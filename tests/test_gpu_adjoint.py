"""GPU parity of the adjoint (dc_stedc_backward / _rank1 / autograd).

Oracle comparisons use sign-invariant cotangents (eigenvectors are defined up
to sign, and each side differentiates its own decomposition): lam_bar, the
loss sum_i c_i (u^T q_i)^2 whose Q_bar = u (2 c o u^T Q)^T flips with q_i,
and Q_bar = R Q S for fixed R, diagonal S.  Bar: relative error of the
gradient vector <= 1e-9 against the dense oracle; <= 1e-6 against central
finite differences (h = 1e-6) of the GPU forward solve.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint, dc
from paper_2008_01990_amd import workloads as W
from tests.gpu_util import announce, cuda, host

pytestmark = pytest.mark.gpu


def _problem(n, seed):
    rng = np.random.default_rng(seed)
    d = 2 + 0.3 * rng.standard_normal(n)
    e = -1 + 0.3 * rng.standard_normal(n - 1)
    return d, e, rng


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("n", [300, 517])
def test_general_adjoint_matches_oracle(lib, n):
    announce(f"adjoint general n={n}")
    d, e, rng = _problem(n, n)
    R = rng.standard_normal((n, n))
    S = rng.standard_normal(n)
    lb = rng.standard_normal(n)
    lo, Qo = dc.eigh_tridiagonal(d, e, leaf=32)
    do, eo = adjoint.backward(lo, Qo, lam_bar=lb, Q_bar=(R @ Qo) * S)
    lam, Q = lib.stedc(cuda(d), cuda(e), leaf=32)
    Qb = (cuda(R) @ Q) * cuda(S)[None, :]
    dg, eg = lib.backward(lam, Q.t().contiguous(), cuda(lb), Qb.t().contiguous())
    assert lib.backward_status() == 0
    assert _rel(host(dg), do) <= 1e-9
    assert _rel(host(eg), eo) <= 1e-9


def test_rank1_matches_general_and_oracle(lib):
    n = 400
    announce("adjoint rank1 n=400")
    d, e, rng = _problem(n, 7)
    w, c, u = rng.standard_normal((3, n))
    lo, Qo = dc.eigh_tridiagonal(d, e, leaf=32)
    ao = u @ Qo
    do, eo = adjoint.backward(lo, Qo, lam_bar=w, Q_bar=np.outer(u, 2 * c * ao))
    lam, Q = lib.stedc(cuda(d), cuda(e), leaf=32)
    a = cuda(u) @ Q
    g = 2 * cuda(c) * a
    d1, e1 = lib.backward_rank1(lam, Q.t().contiguous(), cuda(u), g, lam_bar=cuda(w))
    d2, e2 = lib.backward(lam, Q.t().contiguous(), cuda(w),
                          torch.outer(cuda(u), g).t().contiguous())
    assert _rel(host(d1), host(d2)) <= 1e-12 and _rel(host(e1), host(e2)) <= 1e-12
    assert _rel(host(d1), do) <= 1e-9 and _rel(host(e1), eo) <= 1e-9


def test_hellmann_feynman(lib):
    n = 200
    announce("adjoint hellmann-feynman")
    d, e, rng = _problem(n, 3)
    lb = rng.standard_normal(n)
    lam, Q = lib.stedc(cuda(d), cuda(e), leaf=16)
    dg, eg = lib.backward(lam, Q.t().contiguous(), cuda(lb), None)
    Qh = host(Q)
    assert np.allclose(host(dg), (Qh * Qh) @ lb, rtol=0, atol=1e-13)
    assert np.allclose(host(eg), 2 * (Qh[:-1] * Qh[1:]) @ lb, rtol=0, atol=1e-13)


def test_autograd_against_finite_differences(lib):
    # The adjoint configuration at reduced order: perturbed 1-2-1 matrix,
    # loss sum w_i lam_i + sum c_i (u^T q_i)^2, 32 seeded coordinates.
    P = W.adjoint_problem(n=512, seed=4, n_coords=32)
    n = 512
    announce("adjoint autograd vs FD n=512")
    d = cuda(P["d"]).requires_grad_(True)
    e = cuda(P["e"]).requires_grad_(True)
    w, c, u = cuda(P["w"]), cuda(P["c"]), cuda(P["u"])

    def loss(dd, ee):
        lam, Q = lib.eigh_tridiagonal(dd, ee, leaf=32)
        return (w * lam).sum() + (c * (u @ Q) ** 2).sum()

    L = loss(d, e)
    L.backward()
    grad = torch.cat([d.grad, e.grad]).cpu().numpy()
    h = 1e-6
    fd, ad = [], []
    with torch.no_grad():
        for idx in P["coords"]:
            dp, ep = d.detach().clone(), e.detach().clone()
            dm, em = d.detach().clone(), e.detach().clone()
            if idx < n:
                dp[idx] += h
                dm[idx] -= h
            else:
                ep[idx - n] += h
                em[idx - n] -= h
            fd.append((loss(dp, ep).item() - loss(dm, em).item()) / (2 * h))
            ad.append(grad[idx])
    fd, ad = np.array(fd), np.array(ad)
    assert _rel(ad, fd) <= 1e-6


def test_equal_eigenvalues_set_status_and_warn(lib):
    # The adjoint of a decomposition with two equal eigenvalues has no
    # F_ij = 1 / (lam_j - lam_i) for that pair: the term is dropped and the
    # status word says so (-2000); the autograd backward turns it into a
    # warning.  lam = 1, 2, 2, 3, ... with an orthogonal Q from a QR.
    n = 64
    announce("adjoint equal eigenvalues status")
    rng = np.random.default_rng(9)
    lam = cuda(np.concatenate([[1.0, 2.0, 2.0], 3.0 + np.arange(n - 3)]))
    Q = cuda(np.linalg.qr(rng.standard_normal((n, n)))[0])
    Qbar = cuda(rng.standard_normal((n, n)))
    lib.backward(lam, Q.t().contiguous(), None, Qbar.t().contiguous())
    assert lib.backward_status() == -2000
    assert "equal eigenvalues" in lib.status_string(-2000)
    # distinct eigenvalues: clean status
    lib.backward(lam + cuda(np.arange(n) * 1e-3), Q.t().contiguous(), None,
                 Qbar.t().contiguous())
    assert lib.backward_status() == 0
    # through autograd: a diagonal matrix with a repeated entry has exactly
    # equal eigenvalues, and the backward warns
    d = cuda(np.array([1.0, 2.0, 2.0, 3.0, 5.0])).requires_grad_(True)
    e = cuda(np.zeros(4)).requires_grad_(True)
    lamg, Qg = lib.eigh_tridiagonal(d, e, leaf=32)
    with pytest.warns(RuntimeWarning, match="equal eigenvalues"):
        (Qg.sum(0) ** 2).sum().backward()
