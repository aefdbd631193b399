"""GPU parity of the whole divide-and-conquer solve (dc_stedc_ex).

Bars: eigenvalue error <= 1e-13 ||T||, ||TQ - Q Lambda||_F / (n ||T||) <=
1e-14 and max |Q^T Q - I| <= 1e-12; eigenvalues against the oracle within
1e-13 ||T||; eigenvectors against the oracle entry by entry after sign
alignment, within 100 eps ||T|| / gap_j (an eigenvector is only defined to
that accuracy; tests/parity.py).
"""
import numpy as np
import pytest

from oracle import dc, metrics
from paper_2008_01990_amd import workloads as W
from tests.gpu_util import announce, cuda, host
from tests.parity import assert_eigvecs_match, eigvec_bound

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


def _solve(lib, d, e, **kw):
    lam, Q = lib.stedc(cuda(d), cuda(e), **kw)
    return host(lam), host(Q)


def _check_against_oracle(d, e, lam, Q, leaf):
    lo, Qo = dc.eigh_tridiagonal(d, e, leaf=leaf)
    tn = max(np.abs(lo).max(), 1e-300)
    assert np.abs(lam - lo).max() <= 1e-13 * tn
    assert metrics.orthogonality(Q) <= 1e-12
    assert metrics.residual(d, e, lam, Q) <= 1e-14
    assert_eigvecs_match(Q, Qo, lo, tn)


@pytest.mark.parametrize("n,leaf", [(1024, 32), (777, 16), (200, 64), (65, 32)])
def test_toeplitz_and_ragged_sizes(lib, n, leaf):
    announce(f"stedc toeplitz n={n} leaf={leaf}")
    d, e = W.toeplitz(n)
    lam, Q = _solve(lib, d, e, leaf=leaf)
    k = np.arange(1, n + 1)
    assert metrics.eig_error(lam, 2 - 2 * np.cos(k * np.pi / (n + 1))) <= 1e-13
    _check_against_oracle(d, e, lam, Q, leaf)


def test_toeplitz_sine_vectors_n1024(lib):
    n = 1024
    announce("stedc toeplitz sine vectors n=1024")
    d, e = W.toeplitz(n)
    lam, Q = _solve(lib, d, e, leaf=32)
    k = np.arange(1, n + 1)
    i = np.arange(1, n + 1)[:, None]
    S = np.sqrt(2.0 / (n + 1)) * np.sin(i * k[None, :] * np.pi / (n + 1))
    lam_exact = 2 - 2 * np.cos(k * np.pi / (n + 1))
    err, bound = assert_eigvecs_match(Q, S, lam_exact)
    assert bound.max() < 1e-8          # every column is checked at this size


def test_clement(lib):
    n = 640
    announce(f"stedc clement n={n}")
    d, e = W.clement(n)
    lam, Q = _solve(lib, d, e, leaf=64)
    assert metrics.eig_error(lam, np.arange(-(n - 1), n, 2, dtype=float)) <= 1e-13
    _check_against_oracle(d, e, lam, Q, 64)


@pytest.mark.parametrize("n,seed,leaf", [(500, 0, 32), (129, 1, 8), (2, 2, 1), (1, 3, 32),
                                         (37, 4, 64)])
def test_random(lib, n, seed, leaf):
    announce(f"stedc random n={n} seed={seed} leaf={leaf}")
    rng = np.random.default_rng(seed)
    d, e = W.random_tridiag(n, rng)
    lam, Q = _solve(lib, d, e, leaf=leaf)
    _check_against_oracle(d, e, lam, Q, leaf)


def test_zero_coupling_everything_deflates(lib):
    announce("stedc zero coupling")
    d = np.array([4.0, -2.0, 7.0, 1.0, 1.0, 0.0, -3.0, 5.0] * 8)
    e = np.zeros(63)
    lam, Q = _solve(lib, d, e, leaf=4)
    assert np.array_equal(lam, np.sort(d))
    assert metrics.orthogonality(Q) == 0.0


def test_short_form_and_status(lib):
    announce("stedc short form")
    d, e = W.toeplitz(300)
    lam, Q, st = lib.stedc_short(cuda(d), cuda(e))
    assert st == 0
    k = np.arange(1, 301)
    assert metrics.eig_error(host(lam), 2 - 2 * np.cos(k * np.pi / 301)) <= 1e-13


def test_nonfinite_input_sets_status(lib):
    announce("stedc nan input")
    d, e = W.toeplitz(100)
    d[17] = np.nan
    s = lib.Solver(100, leaf=16)
    s(cuda(d), cuda(e))
    assert s.status() == -1000


def test_hermite_type(lib):
    from scipy.special import roots_hermitenorm
    n = 700
    announce(f"stedc hermite n={n}")
    d, e = W.hermite(n)
    lam, Q = _solve(lib, d, e, leaf=32)
    assert metrics.eig_error(lam, np.sort(roots_hermitenorm(n)[0])) <= 1e-13
    _check_against_oracle(d, e, lam, Q, 32)


def test_sht_matrix(lib):
    n = 1200
    announce(f"stedc sht n={n}")
    d, e = W.sht(n)
    lam, Q = _solve(lib, d, e, leaf=64)
    _check_against_oracle(d, e, lam, Q, 64)


def test_merge_records_count_secular_evaluations(lib):
    # dc_merge_stat's secular counters: every root of a merge is evaluated at
    # least once and at most max_iter + 1 times, so K <= sum <= K * max and
    # 1 <= max <= 201 for every merge with survivors; a merge with none
    # records zeros.  (Random spectra need a few evaluations per root.)
    announce("stedc merge records: secular evaluation counts")
    d, e = W.random_tridiag(3000, np.random.default_rng(21))
    _solve(lib, d, e, leaf=32)
    stats = lib.last_stats()
    assert stats
    total_k = total_it = 0
    for r in stats:
        if r["K"] == 0:
            assert r["sec_iters_sum"] == 0 and r["sec_iters_max"] == 0
            continue
        assert 1 <= r["sec_iters_max"] <= 201
        assert r["K"] <= r["sec_iters_sum"] <= r["K"] * r["sec_iters_max"]
        total_k += r["K"]
        total_it += r["sec_iters_sum"]
    assert 1.0 <= total_it / total_k <= 10.0


@pytest.mark.parametrize("nblocks,delta", [(48, 1e-10), (100, 1e-8)])
def test_glued_wilkinson_rotation_chains(lib, nblocks, delta):
    # Clustered spectra: hundreds of pair rotations per merge, in chains that
    # cross the segments of the parallel deflation walk.
    announce(f"glued wilkinson blocks={nblocks} delta={delta}")
    d, e = W.glued_wilkinson(nblocks, delta)
    lam, Q = _solve(lib, d, e, leaf=32)
    stats = lib.last_stats()
    _check_against_oracle(d, e, lam, Q, 32)
    log = dc.MergeLog()
    dc.eigh_tridiagonal(d, e, leaf=32, log=log)
    ro = sum(r["nrot"] for r in log.records)
    rg = sum(r["nrot"] for r in stats)
    top_g = max(stats, key=lambda r: r["m"])
    # Both sides rotate hundreds of pairs per merge, in chains that cross
    # the walk's segments.  The counts themselves are not compared: in these
    # clusters many rotation tests sit at the deflation tolerance and follow
    # the last bits of the children's spectra and vectors, which two correct
    # root finders do not share.  What is unique, the eigenpairs, is checked
    # above against the oracle.
    assert top_g["nrot"] >= 200 and ro >= 1000 and rg >= 1000, (top_g["nrot"], ro, rg)


@pytest.mark.parametrize("case", ["random", "glued_wilkinson", "clement6000"])
def test_large_solves_against_oracle(lib, case):
    # Merges of 4096 - 8192 rows: the 1024-thread deflation walk and
    # thousands of product tiles per level.  Random and glued-Wilkinson
    # matrices deflate to K ~ 100 - 800 (the glued ones through long rotation
    # chains); Clement n = 6000 keeps K = 3000 at the root and 2689 below it,
    # so its secular, Loewner and scale kernels run three 1024-pole chunks.
    if case == "random":
        d, e = W.random_tridiag(8192, np.random.default_rng(12))
    elif case == "glued_wilkinson":
        d, e = W.glued_wilkinson(390, 1e-10)        # 8190 rows
    else:
        d, e = W.clement(6000)
    d, e = np.asarray(d), np.asarray(e)
    announce(f"stedc large {case} n={len(d)}")
    lam, Q = _solve(lib, d, e, leaf=32)
    _check_against_oracle(d, e, lam, Q, 32)
    if case == "clement6000":
        assert max(r["K"] for r in lib.last_stats()) >= 2048


def test_max_iter_one_reports_non_convergence(lib):
    # A one-iteration cap on the secular root finder: roots stop unconverged
    # and the status word names the first one as a 1-based row position
    # inside the problem (the merge's first row plus the root's index).
    n = 600
    d, e = W.random_tridiag(n, np.random.default_rng(41))
    announce("stedc max_iter=1 status")
    s = lib.Solver(n, leaf=32, max_iter=1)
    s(cuda(d), cuda(e))
    st = s.status()
    assert 1 <= st <= n, st
    assert "did not converge" in lib.status_string(st)
    with pytest.raises(lib.DcError):
        lib.stedc(cuda(d), cuda(e), leaf=32, max_iter=1)
    # the same problem with the default cap converges
    s2 = lib.Solver(n, leaf=32)
    s2(cuda(d), cuda(e))
    assert s2.status() == 0


@pytest.mark.parametrize("k", [-900, -300, 300, 900])
def test_power_of_two_scaling_is_exact(lib, k):
    # Every problem is brought to max(|d|, |e|) in [1, 2) by a power of two
    # before the solve, so T 2^k gives exactly the eigenvalues of T times 2^k
    # and the same eigenvectors, also where the squared pole distances of the
    # secular and scale steps of T 2^k would leave the exponent range.
    rng = np.random.default_rng(31)
    d, e = W.random_tridiag(600, rng)
    announce(f"stedc power-of-two scale 2^{k}")
    lam, Q = _solve(lib, d, e, leaf=32)
    f = 2.0 ** k
    lam_s, Q_s = _solve(lib, d * f, e * f, leaf=32)
    assert np.array_equal(lam_s, lam * f)
    assert np.array_equal(Q_s, Q)


@pytest.mark.parametrize("f", [1e-250, 3e-200, 7e200, 1e250])
def test_tiny_and_huge_norms_meet_the_bars(lib, f):
    # Scales that are not powers of two, near the ends of the exponent range:
    # the bars hold relative to the scale (the oracle solves the unscaled
    # matrix; residual and orthogonality are measured on it).
    d, e = W.clement(500)
    announce(f"stedc clement n=500 scaled by {f:g}")
    lam, Q = _solve(lib, d * f, e * f, leaf=32)
    assert np.all(np.isfinite(lam)) and np.all(np.isfinite(Q))
    lo = np.arange(-499, 500, 2, dtype=float)
    assert metrics.eig_error(lam / f, lo) <= 1e-13
    assert metrics.orthogonality(Q) <= 1e-12
    assert metrics.residual(d, e, lam / f, Q) <= 1e-14


def _structured(case):
    rng = np.random.default_rng(77)
    if case == "graded":                 # eigenvalues from 1 down to about 1e-8
        n = 500
        d = 10.0 ** (-8.0 * np.arange(n) / n)
        e = 0.5 * 10.0 ** (-8.0 * (np.arange(n - 1) + 0.5) / n)
        return d, e, 32
    if case == "zero_couplings":         # rho = 0 at the root and inner tears, and in leaves
        n = 700
        d, e = W.random_tridiag(n, rng)
        e = np.array(e)
        e[[349, 174, 524, 10, 600, 43, 44]] = 0.0
        return d, e, 32
    if case == "constant_tiny":          # every pair deflates at every merge
        n = 640
        return np.full(n, 3.0), 1e-20 * rng.choice([-1.0, 1.0], n - 1), 16
    if case == "wilkinson":              # W_201^+: pairs of nearly equal eigenvalues
        m = 100
        return np.abs(m - np.arange(2 * m + 1)).astype(float), np.ones(2 * m), 32
    if case == "clusters":               # three clusters, couplings 1e-9
        n = 600
        return np.tile([1.0, 2.0, 3.0], n // 3), 1e-9 * rng.standard_normal(n - 1), 32
    if case == "prime_leaf7":
        d, e = W.random_tridiag(997, rng)
        return d, e, 7
    if case == "prime_leaf13":
        d, e = W.random_tridiag(1009, rng)
        return d, e, 13
    raise ValueError(case)


@pytest.mark.parametrize("case", ["graded", "zero_couplings", "constant_tiny", "wilkinson",
                                  "clusters", "prime_leaf7", "prime_leaf13"])
def test_structured_inputs(lib, case):
    d, e, leaf = _structured(case)
    announce(f"stedc structured {case} n={len(d)} leaf={leaf}")
    lam, Q = _solve(lib, d, e, leaf=leaf)
    assert np.all(lam[1:] >= lam[:-1])
    _check_against_oracle(np.asarray(d), np.asarray(e), lam, Q, leaf)


def test_ex_form_captured_in_a_graph(lib):
    # dc_stedc_ex on the plain path allocates nothing and never waits on the
    # host, so it can be captured: the captured solve, replayed three times
    # with other work and synchronisation in between (new inputs before each
    # replay), equals the eager solve of the same inputs bit for bit.
    import torch
    n = 1500
    rng = np.random.default_rng(91)
    s = lib.Solver(n, leaf=32)                   # builds the plan before capture
    d_in = cuda(np.zeros(n))
    e_in = cuda(np.zeros(n - 1))
    dd = torch.empty_like(d_in)
    Qg = torch.empty(n, n, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                # warm-up outside the capture
        dd.copy_(d_in)
        s.solve_into(dd, e_in, Qg)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        dd.copy_(d_in)
        s.solve_into(dd, e_in, Qg)
    for rep in range(3):
        announce(f"stedc_ex graph replay {rep}")
        d, e = W.random_tridiag(n, rng)
        d_in.copy_(cuda(d))
        e_in.copy_(cuda(e))
        scratch = torch.randn(800, 800, dtype=torch.float64, device="cuda")
        float((scratch @ scratch).sum())
        g.replay()
        torch.cuda.synchronize()
        lam_g, Q_g = host(dd).copy(), host(Qg).copy()
        assert s.status() == 0
        lam, Q = _solve(lib, d, e, leaf=32)
        assert np.array_equal(lam_g, lam)
        assert np.array_equal(Q_g.T, Q)              # the buffer holds Q column-major
    _check_against_oracle(np.asarray(d), np.asarray(e), lam, Q, 32)


def test_ex_form_lowrank_captured_in_a_graph(lib):
    # The low-rank path plans on the device (Algorithm 3's switch, the
    # compression, the layouts and task lists of the structured product), so
    # dc_stedc_ex with lr_tol > 0 also allocates nothing and never waits on
    # the host: captured once, replayed with new inputs and other work in
    # between, it equals the eager solve bit for bit.
    import torch
    n = 3000
    kw = dict(leaf=32, lr_tol=1e-10, lr_block=256, lr_min_k=1024)
    rng = np.random.default_rng(93)
    s = lib.Solver(n, **kw)                    # builds the plan and tables before capture
    d_in = cuda(np.zeros(n))
    e_in = cuda(np.zeros(n - 1))
    dd = torch.empty_like(d_in)
    Qg = torch.empty(n, n, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        dd.copy_(d_in)
        s.solve_into(dd, e_in, Qg)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        dd.copy_(d_in)
        s.solve_into(dd, e_in, Qg)
    for rep in range(3):
        announce(f"stedc_ex low-rank graph replay {rep}")
        # perturbed 1-2-1 matrices keep most of every merge (K ~ m)
        d = 2.0 + 1e-3 * rng.standard_normal(n)
        e = -1.0 + 1e-3 * rng.standard_normal(n - 1)
        d_in.copy_(cuda(d))
        e_in.copy_(cuda(e))
        scratch = torch.randn(800, 800, dtype=torch.float64, device="cuda")
        float((scratch @ scratch).sum())
        g.replay()
        torch.cuda.synchronize()
        lam_g, Q_g = host(dd).copy(), host(Qg).copy()
        assert s.status() == 0
        lam, Q = _solve(lib, d, e, **kw)
        assert any(r["path"] == 1 for r in lib.last_stats())
        assert np.array_equal(lam_g, lam)
        assert np.array_equal(Q_g.T, Q)
    assert metrics.orthogonality(Q) <= 1e-9
    assert metrics.residual(d, e, lam, Q) <= 1e-9


def test_concurrent_solves_from_two_threads(lib):
    # Two host threads, each with its own stream and workspace, one on the
    # plain path and one on the low-rank path (per-thread low-rank buffers
    # and host staging), solve repeatedly at the same time; every result
    # equals the same solve run alone, bit for bit.
    import threading
    import torch
    jobs = [(W.random_tridiag(1200, np.random.default_rng(5)), dict(leaf=32)),
            (W.toeplitz(2048), dict(leaf=64, lr_tol=1e-10, lr_block=256, lr_min_k=512))]
    ref = []
    for (d, e), kw in jobs:
        lam, Q = _solve(lib, d, e, **kw)
        ref.append((lam, Q))
    out = [[], []]
    errs = []

    def work(i):
        try:
            (d, e), kw = jobs[i]
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                s = lib.Solver(len(d), **kw)
                for _ in range(4):
                    lam, Q = s(cuda(d), cuda(e))
                    st.synchronize()
                    out[i].append((host(lam).copy(), host(Q).copy(), s.status()))
        except Exception as ex:                  # reported below
            errs.append(repr(ex))

    announce("stedc two threads, plain and low rank")
    th = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not errs, errs
    for i in range(2):
        assert len(out[i]) == 4
        for lam, Q, st in out[i]:
            assert st == 0
            assert np.array_equal(lam, ref[i][0])
            assert np.array_equal(Q, ref[i][1])
