"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

Inputs only: this module builds matrices and generator vectors with the
shapes and value distributions of the paper's workloads and holds none of the
method's arithmetic.

* ``toeplitz``  -- the 1-2-1 Toeplitz-type matrix of Example 2 (d = 2,
                   e = -1; the paper prints off-diagonal +1, which has the
                   same spectrum).
* ``clement``   -- the Clement-type matrix of Example 2 as an n x n matrix:
                   d = 0, e_i = sqrt(i (n - i)), i = 1..n-1.
* ``hermite``   -- the Hermite-type matrix of Example 2: d = 0, e_i = sqrt(i).
* ``sht``       -- the spherical-harmonic-transform matrix of Example 3: row j
                   has diagonal d_{m+2j} and off-diagonal c_{m+2j}, with
                   xi_l = l - m,
                   c_l = sqrt((xi_l+1)(xi_l+2)(l+m+1)(l+m+2) /
                              ((2l+1)(2l+3)^2 (2l+5))),
                   d_l = (2l(l+1) - 2m^2 - 1) / ((2l-1)(2l+3)); m = n by default.
* ``glued_wilkinson`` -- copies of Wilkinson's W_21^+ (d_i = |10 - i|, e = 1)
                   joined by off-diagonal entries delta: tightly clustered
                   eigenvalues, the classic stress case of deflation.
* ``block_cyclic_order`` -- the index order in which a 1-D block-cyclic
                   distribution (block N_B over P process rows) stores a
                   vector: process 0's blocks first, then process 1's, ...
* ``random_tridiag`` / ``batched_sizes`` -- many small problems with
                   d, e ~ U(-1, 1) and sizes log-uniform in [lo, hi].
* ``adjoint_problem`` -- perturbed 1-2-1 matrix plus loss weights w, c, u.
* ``example_cauchy`` -- the Cauchy-like generators of Examples 0 and 1:
                   d_i = i (b - a) / n, w_j = d_j + (b - a) / (2 n), a = 1,
                   b = 9, u, v ~ U(0, 1).
* ``random_secular`` -- a random deflated secular problem (sorted distinct
                   poles, non-negligible z, rho > 0).
"""

import numpy as np


def toeplitz(n):
    return np.full(n, 2.0), np.full(max(n - 1, 0), -1.0)


def clement(n):
    i = np.arange(1, n, dtype=np.float64)
    return np.zeros(n), np.sqrt(i * (n - i))


def hermite(n):
    return np.zeros(n), np.sqrt(np.arange(1, n, dtype=np.float64))


def sht(n, m=None):
    m = n if m is None else m
    l = m + 2 * np.arange(n, dtype=np.float64)
    xi = l - m
    c = np.sqrt((xi + 1) * (xi + 2) * (l + m + 1) * (l + m + 2)
                / ((2 * l + 1) * (2 * l + 3) ** 2 * (2 * l + 5)))
    d = (2 * l * (l + 1) - 2.0 * m * m - 1) / ((2 * l - 1) * (2 * l + 3))
    return d, c[:n - 1].copy()


def random_tridiag(n, rng):
    return rng.uniform(-1.0, 1.0, n), rng.uniform(-1.0, 1.0, max(n - 1, 0))


def batched_sizes(count=256, lo=64, hi=4096, seed=3):
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), count)))
    return sizes.astype(np.int64), rng


def batched_problems(count=256, lo=64, hi=4096, seed=3):
    sizes, rng = batched_sizes(count, lo, hi, seed)
    return [random_tridiag(int(n), rng) for n in sizes]


def adjoint_problem(n=4096, seed=4, n_coords=32):
    rng = np.random.default_rng(seed)
    d = 2.0 + 0.01 * rng.standard_normal(n)
    e = -1.0 + 0.01 * rng.standard_normal(n - 1)
    w = rng.standard_normal(n)
    c = rng.standard_normal(n)
    u = rng.standard_normal(n)
    coords = rng.choice(2 * n - 1, size=n_coords, replace=False)
    return {"d": d, "e": e, "w": w, "c": c, "u": u, "coords": np.sort(coords)}


def example_cauchy(n, seed=0, a=1.0, b=9.0):
    rng = np.random.default_rng(seed)
    i = np.arange(1, n + 1, dtype=np.float64)
    d = i * (b - a) / n
    w = d + (b - a) / (2.0 * n)
    u = rng.uniform(0.0, 1.0, n)
    v = rng.uniform(0.0, 1.0, n)
    return u, v, d, w


def glued_wilkinson(nblocks, delta=1e-10):
    w = np.abs(np.arange(21, dtype=np.float64) - 10.0)
    d = np.tile(w, nblocks)
    e = np.ones(21 * nblocks - 1)
    e[20::21] = delta
    return d, e


def block_cyclic_order(n, nprocs, nb):
    """Global indices in storage order of a block-cyclic layout: block k
    (indices k*nb .. k*nb+nb-1) lives on process k mod nprocs, and each
    process keeps its blocks in increasing order.  nb >= n/nprocs gives the
    contiguous (block) layout, i.e. the identity."""
    blocks = np.arange(n) // nb
    return np.concatenate([np.flatnonzero(blocks % nprocs == p) for p in range(nprocs)])


def random_secular(K, seed=0, spread=1.0, rho=None, cluster=False):
    rng = np.random.default_rng(seed)
    if cluster:
        base = np.sort(rng.uniform(-spread, spread, max(K // 8, 1)))
        D = np.sort(np.concatenate([
            base[rng.integers(0, base.size, K)] + 1e-9 * rng.standard_normal(K)]))
    else:
        D = np.sort(rng.uniform(-spread, spread, K))
    D = np.unique(D)
    while D.size < K:
        D = np.unique(np.concatenate([D, rng.uniform(-spread, spread, K - D.size)]))
    D = np.sort(D)[:K]
    z = rng.uniform(0.1, 1.0, K) * rng.choice([-1.0, 1.0], K)
    z /= np.linalg.norm(z)
    if rho is None:
        rho = float(rng.uniform(0.5, 2.0))
    return D, z, rho


def random_matrix(m, n, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, n))
