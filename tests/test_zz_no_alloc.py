"""The allocation-free rank-one adjoint (dc_stedc_backward_rank1_noalloc)
against the allocating entry point it mirrors, through the C ABI.

Both run the same kernels in the same order on the same inputs, so the
results must be equal bit for bit.  Two calls in a row (the second one
smaller) share the fixed scratch array: the second must not see the first's
contents.  Orders beyond the scratch are rejected on the host.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2008_01990_amd import workloads as W
from tests.gpu_util import announce, cuda

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _case(lib, n, seed):
    P = W.adjoint_problem(n=n, seed=seed, n_coords=4)
    lam, Q = lib.stedc(cuda(P["d"]), cuda(P["e"]), leaf=32)
    Qbuf = Q.t().contiguous()
    u, c, w = cuda(P["u"]), cuda(P["c"]), cuda(P["w"])
    g = 2 * c * (u @ Q)
    return lam, Qbuf, u, g, w


def _noalloc(lib, lam, Qbuf, u, g, w):
    n = lam.numel()
    d_bar = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    e_bar = torch.full((max(n - 1, 1),), np.nan, dtype=torch.float64, device="cuda")
    info = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    L = lib.load()
    rc = L.dc_stedc_backward_rank1_noalloc(n, _ptr(lam), _ptr(Qbuf), Qbuf.shape[1], _ptr(w),
                                           _ptr(u), _ptr(g), _ptr(d_bar), _ptr(e_bar),
                                           _ptr(info), lib._stream())
    assert rc == 0
    torch.cuda.synchronize()
    return d_bar, e_bar[:n - 1], int(info.item())


def test_noalloc_matches_the_allocating_entry_point(lib):
    for n, seed in ((4096, 4), (1500, 5)):          # the second call is smaller
        announce(f"noalloc rank-one adjoint n={n}")
        lam, Qbuf, u, g, w = _case(lib, n, seed)
        d0, e0 = lib.backward_rank1(lam, Qbuf, u, g, lam_bar=w)
        torch.cuda.synchronize()
        d1, e1, st = _noalloc(lib, lam, Qbuf, u, g, w)
        assert st == 0
        assert torch.equal(d1, d0) and torch.equal(e1, e0)


def test_noalloc_limits_and_status(lib):
    L = lib.load()
    assert L.dc_stedc_backward_rank1_noalloc_max_bytes() == 16 << 20
    fake = ctypes.c_void_p(256)
    # beyond the scratch: rejected before any launch
    assert L.dc_stedc_backward_rank1_noalloc(4713, fake, fake, 4713, None, fake, fake, fake,
                                             fake, fake, None) == -1
    assert L.dc_stedc_backward_rank1_noalloc(64, fake, fake, 64, None, fake, fake, fake,
                                             fake, None, None) == -10
    # equal eigenvalues: the caller's status word gets -2000
    announce("noalloc equal eigenvalues")
    n = 64
    rng = np.random.default_rng(3)
    lam = cuda(np.concatenate([[1.0, 2.0, 2.0], 3.0 + np.arange(n - 3)]))
    Qbuf = cuda(np.linalg.qr(rng.standard_normal((n, n)))[0])
    u, g = cuda(rng.standard_normal(n)), cuda(rng.standard_normal(n))
    _, _, st = _noalloc(lib, lam, Qbuf, u, g, None)
    assert st == -2000
