"""The oracle's LU with partial pivoting against its pins (closed forms,
hand-worked cases, ties, exact rational elimination, LAPACK dgetrf,
invariants, singular matrices).  CPU only."""
import numpy as np

import oracle
from lu_piv_pins import failed_lu_piv_pins
from paper_1612_01855_amd import inputs as gen


def test_lu_piv_passes_its_pins():
    assert failed_lu_piv_pins(oracle.lu_piv) == []


def test_lu_piv_thread_count_does_not_change_bits():
    A = gen.rng(21).standard_normal((300, 300))
    L1, U1, p1, _ = oracle.lu_piv(A, nthreads=1)
    L4, U4, p4, _ = oracle.lu_piv(A, nthreads=4)
    assert np.array_equal(p1, p4) and np.array_equal(L1, L4) and np.array_equal(U1, U4)


def test_perm_from_ipiv_composes_the_exchanges():
    assert list(oracle.perm_from_ipiv([2, 2, 2])) == [2, 0, 1]
    assert list(oracle.perm_from_ipiv([0, 1, 2])) == [0, 1, 2]
    A = np.arange(16.0).reshape(4, 4)
    B = A.copy()
    ipiv = [3, 3, 2, 3]
    for j, q in enumerate(ipiv):
        B[[j, q]] = B[[q, j]]
    assert np.array_equal(A[oracle.perm_from_ipiv(ipiv)], B)


def test_lu_piv_rejects_bad_sizes():
    import pytest
    with pytest.raises(ValueError):
        oracle.lu_piv(np.zeros((3, 2)))
    L, U, ipiv, fail = oracle.lu_piv(np.zeros((0, 0)))
    assert L.shape == (0, 0) and len(ipiv) == 0 and fail == -1
