"""The element-wise eigenvector check of the GPU parity tests, on the CPU:
it accepts an independent solver's vectors (LAPACK's MRRR via SciPy against
the oracle) and rejects a single column moved by 1e-6."""
import numpy as np
import pytest
import scipy.linalg

from oracle import dc
from paper_2008_01990_amd import workloads as W
from tests.parity import assert_eigvecs_match


def _pair(n, seed):
    d, e = W.random_tridiag(n, np.random.default_rng(seed))
    lo, Qo = dc.eigh_tridiagonal(d, e, leaf=32)
    ls, Qs = scipy.linalg.eigh_tridiagonal(d, e)
    return lo, Qo, Qs


def test_accepts_an_independent_solver():
    lo, Qo, Qs = _pair(400, 0)
    assert_eigvecs_match(Qs, Qo, lo)
    assert_eigvecs_match(-Qs, Qo, lo)        # sign-free


def test_rejects_a_column_off_by_1e_6():
    lo, Qo, Qs = _pair(400, 1)
    bad = Qs.copy()
    j = int(np.argmax(np.diff(lo, prepend=-np.inf)[1:]))      # a well-separated column
    bad[7, j] += 1e-6
    with pytest.raises(AssertionError):
        assert_eigvecs_match(bad, Qo, lo)
