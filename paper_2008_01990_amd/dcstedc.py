"""Python binding of libdcstedc.so (argument marshalling only).

Every computation runs in the HIP library; this module converts torch
tensors to device pointers and leading dimensions, calls the C ABI on the
current torch stream and raises on a non-zero return code.  There is no CPU
fallback: if the library is missing, importing the handle fails loudly.

Matrices cross the boundary column-major (LAPACK layout).  A torch tensor X
of shape (m, n) is passed as the storage of X.T.contiguous(), and results
come back as the transpose of a row-major (n, ld) buffer.
"""

import ctypes
import os
import warnings

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdcstedc.so")

c_int = ctypes.c_int
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
P = ctypes.c_void_p


class DcOpts(ctypes.Structure):
    _fields_ = [("leaf", c_int), ("lr_tol", c_double), ("lr_block", c_int),
                ("lr_min_k", c_int), ("max_iter", c_int), ("gemm_tile", c_int)]


class MergeStat(ctypes.Structure):
    _fields_ = [("level", c_int), ("m", c_int), ("K", c_int), ("nrot", c_int),
                ("path", c_int), ("flops", c_double), ("lr_blocks", c_int),
                ("lr_rank_sum", c_int), ("lr_rank_max", c_int), ("lr_dense", c_int),
                ("lr_flops_skeleton", c_double), ("lr_flops_fused", c_double),
                ("n1", c_int), ("ntop", c_int), ("nbot", c_int), ("prob", c_int),
                ("sec_iters_sum", c_int), ("sec_iters_max", c_int)]


# (name, restype, argtypes) of every exported entry point.
SIGNATURES = [
    ("dc_opts_default", None, [ctypes.POINTER(DcOpts)]),
    ("dc_stedc", c_int, [c_int, P, P, P, c_int, P]),
    ("dc_stedc_workspace", c_size_t, [c_int, ctypes.POINTER(DcOpts)]),
    ("dc_stedc_ex", c_int, [c_int, P, P, P, c_int, P, c_size_t, P,
                            ctypes.POINTER(DcOpts), P]),
    ("dc_stedc_batched_workspace", c_size_t, [c_int, P, ctypes.POINTER(DcOpts)]),
    ("dc_stedc_batched", c_int, [c_int, P, P, P, P, P, P, c_size_t, P,
                                 ctypes.POINTER(DcOpts), P]),
    ("dc_secular", c_int, [c_int, P, P, c_double, P, P, P, P, P, c_int, P]),
    ("dc_merge_update", c_int, [c_int, c_int, P, c_int, P, P, P, P, P, P, c_int,
                                c_double, c_int, P]),
    ("dc_merge_lowrank_ranks", c_int, [c_int, P, P, P, P, P, c_double, c_int, c_int, P, P]),
    ("dc_autotune", c_int, [c_int, P]),
    ("dc_autotune_table", c_int, [P, c_int]),
    ("dc_autotune_batched", c_int, [c_int, P, P, P, P, P, P, c_size_t, P,
                                    ctypes.POINTER(DcOpts), P]),
    ("dc_autotune_levels", c_int, [c_int, P, c_int, P, c_int]),
    ("dc_autotune_lowrank", c_int, [c_int, P, c_int, P, P]),
    ("dc_stedc_backward", c_int, [c_int, P, P, c_int, P, P, c_int, P, P, P]),
    ("dc_stedc_backward_workspace", c_size_t, [c_int, c_int]),
    ("dc_stedc_backward_ex", c_int, [c_int, P, P, c_int, P, P, c_int, P, P, P, c_size_t, P,
                                     P]),
    ("dc_stedc_backward_rank1", c_int, [c_int, P, P, c_int, P, P, P, P, P, P]),
    ("dc_stedc_backward_rank1_noalloc", c_int, [c_int, P, P, c_int, P, P, P, P, P, P, P]),
    ("dc_stedc_backward_rank1_noalloc_max_bytes", c_size_t, []),
    ("dc_last_info", c_int, [P]),
    ("dc_strerror", ctypes.c_char_p, [c_int]),
    ("dc_status_string", ctypes.c_char_p, [c_int]),
    ("dc_last_stats", c_int, [ctypes.POINTER(MergeStat), c_int]),
    ("dc_profile_enable", c_int, [c_int]),
    ("dc_profile_read", c_int, [P, c_int]),
    ("dc_profile_read_lowrank", c_int, [P, c_int]),
]

# Extra (non-header) hooks used by tests and the benchmark.
EXTRA = [
    ("dc_stedc_batched_eager", c_int, [c_int, P, P, P, P, P, P, c_size_t, P,
                                       ctypes.POINTER(DcOpts), P]),
    ("dc_merge_update_variant", c_int, [c_int, c_int, P, c_int, P, P, P, P, P, P,
                                        c_int, c_int, P]),
]

_lib = None


def load():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2008_01990_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES + EXTRA:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class DcError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        msg = load().dc_strerror(rc).decode()
        raise DcError(f"{what} returned {rc}: {msg}")


def status_string(status):
    """Text of a device status word (dc_status_string)."""
    return load().dc_status_string(int(status)).decode()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype=torch.float64):
    t = torch.as_tensor(t)
    return t.to(device="cuda", dtype=dtype).contiguous()


def opts(leaf=32, lr_tol=0.0, lr_block=0, lr_min_k=0, max_iter=200, gemm_tile=0):
    o = DcOpts()
    load().dc_opts_default(ctypes.byref(o))
    o.leaf, o.lr_tol, o.lr_block = leaf, lr_tol, lr_block
    o.lr_min_k, o.max_iter, o.gemm_tile = lr_min_k, max_iter, gemm_tile
    return o


def to_colmajor(X):
    """(m, n) tensor -> contiguous storage of its column-major layout."""
    return X.t().contiguous()


def from_colmajor(buf, m):
    """Row-major (n, ld) buffer holding a column-major m x n matrix -> (m, n) view."""
    return buf[:, :m].t()


class Solver:
    """Reusable workspace for repeated solves of one order n."""

    def __init__(self, n, **kw):
        self.n = n
        self.o = opts(**kw)
        lib = load()
        self.lwork = lib.dc_stedc_workspace(n, ctypes.byref(self.o))
        if self.lwork == 0 and n > 0:
            raise DcError("dc_stedc_workspace failed")
        self.work = torch.empty(max(self.lwork, 256) // 8 + 32, dtype=torch.float64,
                                device="cuda")
        self.info = torch.zeros(1, dtype=torch.int32, device="cuda")

    def _wptr(self):
        addr = self.work.data_ptr()
        return ctypes.c_void_p((addr + 255) & ~255)

    def solve_into(self, d, e, Qbuf):
        """In place: d -> eigenvalues, Qbuf (n, n) row-major = Q column-major."""
        n = self.n
        rc = load().dc_stedc_ex(n, _ptr(d), _ptr(e), _ptr(Qbuf), n, self._wptr(),
                                self.lwork, _ptr(self.info), ctypes.byref(self.o),
                                _stream())
        _check(rc, "dc_stedc_ex")

    def autotune_on(self, d, e, Qbuf):
        """Per-level tile choice measured on this problem (dc_autotune_batched
        with one problem); d and e are left as given, Qbuf is scratch.
        Returns the chosen variant per level, deepest first."""
        lib = load()
        n_host = (ctypes.c_int * 1)(self.n)
        Pp = ctypes.c_void_p
        dp, ep, qp = (Pp * 1)(d.data_ptr()), (Pp * 1)(e.data_ptr()), (Pp * 1)(Qbuf.data_ptr())
        ldq = (ctypes.c_int * 1)(max(self.n, 1))
        rc = lib.dc_autotune_batched(1, n_host, dp, ep, qp, ldq, self._wptr(), self.lwork,
                                     _ptr(self.info), ctypes.byref(self.o), _stream())
        _check(rc, "dc_autotune_batched")
        nl = lib.dc_autotune_levels(1, n_host, self.o.leaf, None, 0)
        out = (ctypes.c_int * max(nl, 1))()
        lib.dc_autotune_levels(1, n_host, self.o.leaf, ctypes.cast(out, ctypes.c_void_p), nl)
        return list(out)[:nl]

    def tuned_lowrank(self):
        """(block, min_k) that autotune_on chose for this size with lr_tol > 0,
        or None."""
        n_host = (ctypes.c_int * 1)(self.n)
        b, k = ctypes.c_int(0), ctypes.c_int(0)
        r = load().dc_autotune_lowrank(1, n_host, self.o.leaf, ctypes.byref(b), ctypes.byref(k))
        return (b.value, k.value) if r == 1 else None

    def __call__(self, d, e):
        d = _dev(d).clone()
        e = _dev(e).clone() if self.n > 1 else torch.zeros(1, dtype=torch.float64,
                                                            device="cuda")
        Qbuf = torch.empty(max(self.n, 1), max(self.n, 1), dtype=torch.float64,
                           device="cuda")
        self.solve_into(d, e, Qbuf)
        return d, from_colmajor(Qbuf, self.n)

    def status(self):
        return int(self.info.item())


def stedc(d, e, **kw):
    """(lam ascending, Q) of T(d, e) on the GPU; Q is an (n, n) view."""
    n = int(torch.as_tensor(d).numel())
    s = Solver(n, **kw)
    lam, Q = s(d, e)
    st = s.status()
    if st != 0:
        raise DcError(f"device status {st}: {status_string(st)}")
    return lam, Q


def stedc_short(d, e):
    """The short form dc_stedc (library-allocated workspace)."""
    n = int(torch.as_tensor(d).numel())
    d = _dev(d).clone()
    e = _dev(e).clone() if n > 1 else torch.zeros(1, dtype=torch.float64, device="cuda")
    Qbuf = torch.empty(max(n, 1), max(n, 1), dtype=torch.float64, device="cuda")
    _check(load().dc_stedc(n, _ptr(d), _ptr(e), _ptr(Qbuf), max(n, 1), _stream()),
           "dc_stedc")
    st = load().dc_last_info(_stream())
    return d, from_colmajor(Qbuf, n), st


def last_stats():
    lib = load()
    cnt = lib.dc_last_stats(None, 0)
    arr = (MergeStat * max(cnt, 1))()
    lib.dc_last_stats(arr, cnt)
    return [dict(level=r.level, m=r.m, K=r.K, nrot=r.nrot, path=r.path, flops=r.flops,
                 lr_blocks=r.lr_blocks, lr_rank_sum=r.lr_rank_sum, lr_rank_max=r.lr_rank_max,
                 lr_dense=r.lr_dense, lr_flops_skeleton=r.lr_flops_skeleton,
                 lr_flops_fused=r.lr_flops_fused, n1=r.n1, ntop=r.ntop, nbot=r.nbot,
                 prob=r.prob, sec_iters_sum=r.sec_iters_sum,
                 sec_iters_max=r.sec_iters_max) for r in arr[:cnt]]


PHASES = ("deflate", "rotate", "secular", "assemble", "product", "copy")


def profile_enable(on=True):
    load().dc_profile_enable(1 if on else 0)


def profile_read():
    """Per level (deepest first): dict of phase -> milliseconds."""
    lib = load()
    nl = lib.dc_profile_read(None, 0)
    buf = (ctypes.c_double * max(6 * nl, 1))()
    lib.dc_profile_read(ctypes.cast(buf, ctypes.c_void_p), 6 * nl)
    return [dict(zip(PHASES, buf[6 * i:6 * i + 6])) for i in range(nl)]


LR_PHASES = ("compress", "skeleton", "fused")


def profile_read_lowrank():
    """Per level (deepest first): dict of low-rank stage -> milliseconds
    (0 on levels without a low-rank merge)."""
    lib = load()
    nl = lib.dc_profile_read_lowrank(None, 0)
    buf = (ctypes.c_double * max(3 * nl, 1))()
    lib.dc_profile_read_lowrank(ctypes.cast(buf, ctypes.c_void_p), 3 * nl)
    return [dict(zip(LR_PHASES, buf[3 * i:3 * i + 3])) for i in range(nl)]


def secular(D, z, rho, max_iter=200):
    """(org, tau, zhat, scale) of diag(D) + rho z z^T."""
    D = _dev(D)
    z = _dev(z)
    K = D.numel()
    org = torch.empty(K, dtype=torch.int32, device="cuda")
    tau = torch.empty(K, dtype=torch.float64, device="cuda")
    zhat = torch.empty_like(tau)
    scale = torch.empty_like(tau)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    _check(load().dc_secular(K, _ptr(D), _ptr(z), float(rho), _ptr(org), _ptr(tau),
                             _ptr(zhat), _ptr(scale), _ptr(info), max_iter, _stream()),
           "dc_secular")
    st = int(info.item())
    if st != 0:
        raise DcError(f"dc_secular device status {st}: {status_string(st)}")
    return org, tau, zhat, scale


def autotune(max_n):
    """Time the product tile variants per level size on this device; returns
    the chosen variant per size bucket (bucket b: largest merge in
    (2^(b-1), 2^b])."""
    _check(load().dc_autotune(int(max_n), _stream()), "dc_autotune")
    return autotune_table()


def autotune_table():
    lib = load()
    nb = lib.dc_autotune_table(None, 0)
    out = (ctypes.c_int * nb)()
    lib.dc_autotune_table(ctypes.cast(out, ctypes.c_void_p), nb)
    return list(out)


def merge_lowrank_ranks(Dbar, org, tau, zhat, scale, lr_tol, lr_block, rank_cap=0):
    """Block ranks (nb x nb numpy array, -1 diagonal, -2 above the cap).

    rank_cap 0 gives the ranks the low-rank product uses (cap min(128, b/2));
    rank_cap > 0 counts ranks up to that cap without forming the factors.
    """
    import numpy as np
    K = Dbar.numel()
    nb = (K + lr_block - 1) // lr_block
    out = (ctypes.c_int * (nb * nb))()
    _check(load().dc_merge_lowrank_ranks(K, _ptr(Dbar), _ptr(org), _ptr(tau), _ptr(zhat),
                                         _ptr(scale), float(lr_tol), int(lr_block),
                                         int(rank_cap), ctypes.cast(out, ctypes.c_void_p),
                                         _stream()),
           "dc_merge_lowrank_ranks")
    return np.array(out[:], dtype=np.int64).reshape(nb, nb)


def merge_update(Qnd_cm, m, K, Dbar, org, tau, zhat, scale, lr_tol=0.0, lr_block=0,
                 ldq=None, out=None, variant=None):
    """C = Qnd U with U generated from (Dbar, org, tau, zhat, scale).

    Qnd_cm is the column-major storage of Qnd: a tensor of shape (K, ldq).
    Returns the column-major storage of C, shape (K, m).
    """
    ldq = ldq if ldq is not None else Qnd_cm.shape[1]
    C = out if out is not None else torch.empty(K, m, dtype=torch.float64, device="cuda")
    args = (m, K, _ptr(Qnd_cm), ldq, _ptr(Dbar), _ptr(org), _ptr(tau), _ptr(zhat),
            _ptr(scale), _ptr(C), C.shape[1])
    if variant is not None:
        _check(load().dc_merge_update_variant(*args, variant, _stream()),
               "dc_merge_update_variant")
    else:
        _check(load().dc_merge_update(*args, float(lr_tol), int(lr_block), _stream()),
               "dc_merge_update")
    return C


def backward(lam, Qbuf, lam_bar=None, Qbar_cm=None):
    """(d_bar, e_bar) of (lam, Q) = eig(T); Qbuf / Qbar_cm are column-major
    storages ((n, ld) row-major buffers)."""
    n = lam.numel()
    d_bar = torch.empty(n, dtype=torch.float64, device="cuda")
    e_bar = torch.empty(max(n - 1, 1), dtype=torch.float64, device="cuda")
    _check(load().dc_stedc_backward(n, _ptr(lam), _ptr(Qbuf), Qbuf.shape[1],
                                    _ptr(lam_bar), _ptr(Qbar_cm),
                                    Qbar_cm.shape[1] if Qbar_cm is not None else n,
                                    _ptr(d_bar), _ptr(e_bar), _stream()),
           "dc_stedc_backward")
    return d_bar, e_bar[:max(n - 1, 0)]


def backward_workspace(n, with_qbar):
    """Workspace tensor (float64, on the GPU) for backward_ex, with room to
    align its start to 256 bytes."""
    nbytes = load().dc_stedc_backward_workspace(n, 1 if with_qbar else 0)
    return torch.empty(max(nbytes, 8) // 8 + 33, dtype=torch.float64, device="cuda")


def backward_ex(lam, Qbuf, lam_bar=None, Qbar_cm=None, work=None, info=None, d_bar=None,
                e_bar=None):
    """dc_stedc_backward_ex: the same gradient with caller workspace and device
    status (info, an int32 tensor of one element); allocates nothing itself
    when work, info and the outputs are given (capturable).  Returns
    (d_bar, e_bar, info)."""
    n = lam.numel()
    if work is None:
        work = backward_workspace(n, Qbar_cm is not None)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
    if d_bar is None:
        d_bar = torch.empty(n, dtype=torch.float64, device="cuda")
    if e_bar is None:
        e_bar = torch.empty(max(n - 1, 1), dtype=torch.float64, device="cuda")
    addr = work.data_ptr()
    start = (addr + 255) & ~255
    _check(load().dc_stedc_backward_ex(n, _ptr(lam), _ptr(Qbuf), Qbuf.shape[1],
                                       _ptr(lam_bar), _ptr(Qbar_cm),
                                       Qbar_cm.shape[1] if Qbar_cm is not None else n,
                                       _ptr(d_bar), _ptr(e_bar), ctypes.c_void_p(start),
                                       work.numel() * 8 - (start - addr), _ptr(info),
                                       _stream()),
           "dc_stedc_backward_ex")
    return d_bar, e_bar[:max(n - 1, 0)], info


def backward_rank1(lam, Qbuf, u, g, lam_bar=None):
    """Gradient for Q_bar = u g^T (rank one)."""
    n = lam.numel()
    d_bar = torch.empty(n, dtype=torch.float64, device="cuda")
    e_bar = torch.empty(max(n - 1, 1), dtype=torch.float64, device="cuda")
    _check(load().dc_stedc_backward_rank1(n, _ptr(lam), _ptr(Qbuf), Qbuf.shape[1],
                                          _ptr(lam_bar), _ptr(_dev(u)), _ptr(_dev(g)),
                                          _ptr(d_bar), _ptr(e_bar), _stream()),
           "dc_stedc_backward_rank1")
    return d_bar, e_bar[:max(n - 1, 0)]


def backward_status():
    """Status word of the last backward call on the current stream."""
    return load().dc_last_info(_stream())


class EighTridiagonal(torch.autograd.Function):
    """(lam, Q) = eig(T(d, e)) with the library's adjoint as backward.

    forward: dc_stedc_ex; backward: dc_stedc_backward_ex on the saved final
    (lam, Q) only -- no per-level state is kept.
    """

    @staticmethod
    def forward(ctx, d, e, leaf=32, lr_tol=0.0, lr_block=0, lr_min_k=0):
        n = d.numel()
        s = Solver(n, leaf=leaf, lr_tol=lr_tol, lr_block=lr_block, lr_min_k=lr_min_k)
        lam = d.detach().to("cuda", torch.float64).clone().contiguous()
        ee = (e.detach().to("cuda", torch.float64).clone().contiguous() if n > 1
              else torch.zeros(1, dtype=torch.float64, device="cuda"))
        Qbuf = torch.empty(max(n, 1), max(n, 1), dtype=torch.float64, device="cuda")
        s.solve_into(lam, ee, Qbuf)
        st = s.status()
        if st != 0:
            raise DcError(f"device status {st}: {status_string(st)}")
        ctx.save_for_backward(lam, Qbuf)
        return lam.clone(), from_colmajor(Qbuf, n)

    @staticmethod
    def backward(ctx, lam_bar, Q_bar):
        lam, Qbuf = ctx.saved_tensors
        lb = lam_bar.contiguous() if lam_bar is not None else None
        qb = Q_bar.t().contiguous() if Q_bar is not None else None
        d_bar, e_bar, info = backward_ex(lam, Qbuf, lb, qb)
        st = int(info.item())                  # waits for the backward kernels
        if st == -2000:
            warnings.warn("eigh_tridiagonal backward: equal eigenvalues, the terms "
                          "1 / (lam_j - lam_i) of such pairs were dropped "
                          "(the gradient is not defined there)", RuntimeWarning)
        elif st != 0:
            raise DcError(f"dc_stedc_backward device status {st}: {status_string(st)}")
        return d_bar, e_bar, None, None, None, None


def eigh_tridiagonal(d, e, **kw):
    """Differentiable (lam ascending, Q) of the symmetric tridiagonal T(d, e)."""
    return EighTridiagonal.apply(d, e, *[kw.get(k, v) for k, v in
                                         (("leaf", 32), ("lr_tol", 0.0), ("lr_block", 0),
                                          ("lr_min_k", 0))])


class BatchedSolver:
    """Workspace and pointer tables for one batch of tridiagonal problems.

    solve() runs dc_stedc_batched (level schedule replayed as a HIP graph);
    solve(graph=False) runs the same schedule eagerly.
    """

    def __init__(self, sizes, leaf=32, gemm_tile=0, lr_tol=0.0, lr_block=0, lr_min_k=0):
        self.sizes = [int(v) for v in sizes]
        self.count = len(self.sizes)
        self.o = opts(leaf=leaf, gemm_tile=gemm_tile, lr_tol=lr_tol, lr_block=lr_block,
                      lr_min_k=lr_min_k)
        lib = load()
        self.n_host = (ctypes.c_int * max(self.count, 1))(*self.sizes)
        self.lwork = lib.dc_stedc_batched_workspace(self.count, self.n_host,
                                                    ctypes.byref(self.o))
        if self.lwork == 0 and self.count > 0:
            raise DcError("dc_stedc_batched_workspace failed")
        self.work = torch.empty(max(self.lwork, 256) // 8 + 32, dtype=torch.float64,
                                device="cuda")
        self.info = torch.zeros(max(self.count, 1), dtype=torch.int32, device="cuda")
        self.d = [torch.zeros(max(n, 1), dtype=torch.float64, device="cuda") for n in self.sizes]
        self.e = [torch.zeros(max(n - 1, 1), dtype=torch.float64, device="cuda")
                  for n in self.sizes]
        self.Q = [torch.empty(max(n, 1), max(n, 1), dtype=torch.float64, device="cuda")
                  for n in self.sizes]
        P = ctypes.c_void_p
        self.dp = (P * max(self.count, 1))(*[t.data_ptr() for t in self.d])
        self.ep = (P * max(self.count, 1))(*[t.data_ptr() for t in self.e])
        self.qp = (P * max(self.count, 1))(*[t.data_ptr() for t in self.Q])
        self.ldq = (ctypes.c_int * max(self.count, 1))(*[max(n, 1) for n in self.sizes])

    def load_inputs(self, problems):
        """Copy the problems' (d, e) into the device buffers.

        A device copy of the diagonals is kept so that restore() can put
        them back after a solve (the solve overwrites d with eigenvalues;
        e is only read).
        """
        for i, (d, e) in enumerate(problems):
            n = self.sizes[i]
            if n:
                self.d[i][:n].copy_(torch.as_tensor(d))
            if n > 1:
                self.e[i][:n - 1].copy_(torch.as_tensor(e))
        self.d_saved = [t.clone() for t in self.d]

    def restore(self):
        """Put back the diagonals given to the last load_inputs (device copy)."""
        torch._foreach_copy_(self.d, self.d_saved)

    def solve(self, graph=True):
        lib = load()
        fn = lib.dc_stedc_batched if graph else lib.dc_stedc_batched_eager
        addr = self.work.data_ptr()
        rc = fn(self.count, self.n_host, self.dp, self.ep, self.qp, self.ldq,
                ctypes.c_void_p((addr + 255) & ~255), self.lwork, _ptr(self.info),
                ctypes.byref(self.o), _stream())
        _check(rc, "dc_stedc_batched")

    def autotune(self):
        """Measure the product tile variants on this batch's loaded inputs and
        keep the fastest per level (dc_autotune_batched); returns the chosen
        variant per level, deepest first.  d and e are left as loaded."""
        lib = load()
        addr = self.work.data_ptr()
        rc = lib.dc_autotune_batched(self.count, self.n_host, self.dp, self.ep, self.qp,
                                     self.ldq, ctypes.c_void_p((addr + 255) & ~255),
                                     self.lwork, _ptr(self.info), ctypes.byref(self.o),
                                     _stream())
        _check(rc, "dc_autotune_batched")
        return self.tuned_levels()

    def tuned_lowrank(self):
        """(block, min_k) chosen for this batch by autotune() with lr_tol > 0,
        or None."""
        b, k = ctypes.c_int(0), ctypes.c_int(0)
        r = load().dc_autotune_lowrank(self.count, self.n_host, self.o.leaf, ctypes.byref(b),
                                       ctypes.byref(k))
        return (b.value, k.value) if r == 1 else None

    def tuned_levels(self):
        lib = load()
        nl = lib.dc_autotune_levels(self.count, self.n_host, self.o.leaf, None, 0)
        out = (ctypes.c_int * max(nl, 1))()
        lib.dc_autotune_levels(self.count, self.n_host, self.o.leaf,
                               ctypes.cast(out, ctypes.c_void_p), nl)
        return list(out)[:nl]

    def result(self, i):
        n = self.sizes[i]
        return self.d[i][:n], from_colmajor(self.Q[i], n)

    def status(self):
        return self.info[:self.count].cpu().tolist()
