"""GPU parity of the adjoint (dc_stedc_backward / _rank1 / autograd).

Oracle comparisons use sign-invariant cotangents (eigenvectors are defined up
to sign, and each side differentiates its own decomposition): lam_bar, the
loss sum_i c_i (u^T q_i)^2 whose Q_bar = u (2 c o u^T Q)^T flips with q_i,
and Q_bar = R Q S for fixed R, diagonal S.  Bar: relative error of the
gradient vector <= 1e-9 against the dense oracle; <= 1e-6 against central
finite differences (h = 1e-6) of the GPU forward solve.
"""
import ctypes

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


@pytest.mark.parametrize("n", [40, 517, 1030])
def test_backward_ex_matches_short_form_and_oracle(lib, n):
    # dc_stedc_backward_ex (caller workspace, device status) gives the short
    # form's result bit for bit; n = 40 takes the small-matrix product,
    # 517 and 1030 ragged edges of the TN tiles and of the 8-wide k chunks.
    announce(f"adjoint backward_ex n={n}")
    d, e, rng = _problem(n, 100 + n)
    R = rng.standard_normal((n, n))
    S = rng.standard_normal(n)
    lb = rng.standard_normal(n)
    lam, Q = lib.stedc(cuda(d), cuda(e), leaf=32)
    Qb = (cuda(R) @ Q) * cuda(S)[None, :]
    Qbuf, Qbar_cm = Q.t().contiguous(), Qb.t().contiguous()
    d1, e1 = lib.backward(lam, Qbuf, cuda(lb), Qbar_cm)
    d2, e2, info = lib.backward_ex(lam, Qbuf, cuda(lb), Qbar_cm)
    torch.cuda.synchronize()
    assert int(info.item()) == 0 and lib.backward_status() == 0
    assert torch.equal(d1, d2) and torch.equal(e1, e2)
    lo, Qo = dc.eigh_tridiagonal(d, e, leaf=32)
    do, eo = adjoint.backward(lo, Qo, lam_bar=lb, Q_bar=(R @ Qo) * S)
    assert _rel(host(d2), do) <= 1e-9 and _rel(host(e2), eo) <= 1e-9


def test_backward_ex_rejects_bad_workspace(lib):
    n = 64
    lam = torch.linspace(0, 1, n, dtype=torch.float64, device="cuda")
    Qbuf = torch.eye(n, dtype=torch.float64, device="cuda")
    need = lib.load().dc_stedc_backward_workspace(n, 1)
    work = torch.empty(need // 8 + 64, dtype=torch.float64, device="cuda")
    start = (work.data_ptr() + 255) & ~255
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    P = ctypes.c_void_p
    args = lambda w, lw, inf: (n, P(lam.data_ptr()), P(Qbuf.data_ptr()), n, None,
                               P(Qbuf.data_ptr()), n, P(out.data_ptr()), P(out.data_ptr()),
                               w, lw, inf, None)
    f = lib.load().dc_stedc_backward_ex
    assert f(*args(P(start + 8), need, P(info.data_ptr()))) == -10
    assert f(*args(P(start), need - 8, P(info.data_ptr()))) == -11
    assert f(*args(P(start), need, None)) == -12


def test_backward_ex_captured_in_a_graph(lib):
    # The _ex form allocates nothing and never waits: captured once, its
    # replays (with eager work and synchronisations between them) give the
    # eager result bit for bit.
    n = 700
    announce("adjoint backward_ex graph capture")
    d, e, rng = _problem(n, 31)
    lam, Q = lib.stedc(cuda(d), cuda(e), leaf=32)
    Qbuf = Q.t().contiguous()
    Qbar_cm = (cuda(rng.standard_normal((n, n))) @ Q).t().contiguous()
    lb = cuda(rng.standard_normal(n))
    work = lib.backward_workspace(n, True)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    d_out = torch.empty(n, dtype=torch.float64, device="cuda")
    e_out = torch.empty(n, dtype=torch.float64, device="cuda")
    d_ref, e_ref, _ = lib.backward_ex(lam, Qbuf, lb, Qbar_cm, work=work, info=info)
    d_ref, e_ref = d_ref.clone(), e_ref.clone()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        lib.backward_ex(lam, Qbuf, lb, Qbar_cm, work=work, info=info, d_bar=d_out,
                        e_bar=e_out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        lib.backward_ex(lam, Qbuf, lb, Qbar_cm, work=work, info=info, d_bar=d_out,
                        e_bar=e_out)
    for rep in range(3):
        d_out.zero_()
        e_out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        assert torch.equal(d_out, d_ref), rep
        assert torch.equal(e_out[:n - 1], e_ref), rep


def test_unsorted_eigenvalues_take_the_general_instance(lib):
    # The gradient does not depend on the order of the eigenpairs.  Permuted
    # (lam, Q, lam_bar, Q_bar) are not increasing, so the band product runs
    # its instance with the equality test (and finds no equal pair): same
    # gradient up to the order of the sums, status 0.
    n = 333
    announce("adjoint unsorted eigenvalues")
    d, e, rng = _problem(n, 77)
    lam, Q = lib.stedc(cuda(d), cuda(e), leaf=32)
    lb = cuda(rng.standard_normal(n))
    Qb = cuda(rng.standard_normal((n, n))) @ Q
    d1, e1, info1 = lib.backward_ex(lam, Q.t().contiguous(), lb, Qb.t().contiguous())
    perm = torch.as_tensor(rng.permutation(n), device="cuda")
    d2, e2, info2 = lib.backward_ex(lam[perm].contiguous(), Q[:, perm].t().contiguous(),
                                    lb[perm].contiguous(), Qb[:, perm].t().contiguous())
    torch.cuda.synchronize()
    assert int(info1.item()) == 0 and int(info2.item()) == 0
    assert _rel(host(d2), host(d1)) <= 1e-12 and _rel(host(e2), host(e1)) <= 1e-12
