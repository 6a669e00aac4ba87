"""Pins of the Cholesky oracle, A = L L^T by the column-by-column definition
(the factorization whose panel step is a triangular solve with many
right-hand sides), and planted mistakes in it that the pins must catch.  CPU
only.

Exact pins: for an integer lower-triangular L with positive diagonal, A = L
L^T has integer entries, every intermediate of the definition is an integer
far below 2^53, and the square roots are of perfect squares, so the oracle
must return L bit for bit; the symmetric Pascal matrix C(i+j, i) is the
special case whose factor is the lower Pascal matrix C(i, j).  Closed forms:
diag(d) gives sqrt(d); the second-difference matrix tridiag(-1, 2, -1) has
l_ii = sqrt((i+2)/(i+1)) and l_{i+1,i} = -sqrt((i+1)/(i+2)) (0-based).  A
library routine: LAPACK's factor through numpy.  Invariants: the backward
error bound |A - L L^T| <= gamma_{n+1} |L| |L^T| and the failure index of a
matrix that is not positive definite."""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1612_01855_amd import inputs as gen

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
U = 2.0 ** -53


def _nan_upper(A):
    A = np.array(A, dtype=np.float64)
    A[np.triu_indices(A.shape[0], 1)] = np.nan
    return A


def _int_spd(n, seed):
    L = gen.int_lower_positive(n, seed)
    Li = L.astype(np.int64)
    return L, (Li @ Li.T).astype(np.float64)


def _pascal(n):
    A = np.array([[math.comb(i + j, i) for j in range(n)] for i in range(n)], dtype=np.float64)
    L = np.array([[math.comb(i, j) if j <= i else 0 for j in range(n)] for i in range(n)],
                 dtype=np.float64)
    return A, L


def _failed_pins(chol):
    failed = []
    L0, A = _int_spd(14, 3)
    L, f = chol(_nan_upper(A))
    if f != -1 or not np.array_equal(L, L0):
        failed.append("integer_factor")
    A, Lp = _pascal(16)
    L, f = chol(_nan_upper(A))
    if f != -1 or not np.array_equal(L, Lp):
        failed.append("pascal")
    d = gen.rng(5).uniform(0.5, 4.0, size=9)
    L, f = chol(_nan_upper(np.diag(d)))
    if f != -1 or not np.array_equal(L, np.diag(np.sqrt(d))):
        failed.append("diagonal")
    n = 40
    T = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    L, f = chol(_nan_upper(T))
    i = np.arange(n, dtype=np.float64)
    E = np.diag(np.sqrt((i + 2) / (i + 1))) - np.diag(np.sqrt((i[:-1] + 1) / (i[:-1] + 2)), -1)
    if f != -1 or not np.allclose(L, E, rtol=8 * U, atol=0):
        failed.append("second_difference")
    L0, A = _int_spd(10, 8)
    A[6, 6] -= L0[6, 6] ** 2 + 1.0      # pivot 6 becomes -1; pivots 0..5 unchanged
    L, f = chol(_nan_upper(A))
    if f != 6 or not np.array_equal(L[:6, :6], L0[:6, :6]):
        failed.append("failure_index")
    return failed


def test_oracle_passes_its_pins():
    assert _failed_pins(oracle.chol) == []


@pytest.mark.parametrize("n", [1, 37, 300])
def test_agrees_with_lapack(n):
    A = gen.spd(n, n + 1)
    L, f = oracle.chol(A)
    assert f == -1
    assert oracle.rel_fro_err(L, np.linalg.cholesky(A)) <= 1e-14


@pytest.mark.parametrize("n,m", [(400, 800), (257, 64)])
def test_backward_error_bound(n, m):
    A = gen.spd(n, 11, m=m)
    L, f = oracle.chol(A)
    assert f == -1
    gamma = (n + 1) * U / (1 - (n + 1) * U)
    assert np.all(np.abs(A - L @ L.T) <= gamma * (np.abs(L) @ np.abs(L.T)))


def test_zero_and_nan_pivots():
    L0, A = _int_spd(9, 2)
    Z = A.copy()
    Z[4, 4] -= L0[4, 4] ** 2              # pivot 4 is exactly zero
    assert oracle.chol(Z)[1] == 4
    N = A.copy()
    N[7, 7] = np.nan
    assert oracle.chol(N)[1] == 7
    assert oracle.chol(-np.eye(3))[1] == 0


def test_threads_are_bitwise_and_upper_unread():
    A = gen.spd(600, 4)
    L1, _ = oracle.chol(A, nthreads=1)
    L8, _ = oracle.chol(_nan_upper(A), nthreads=8)
    assert np.array_equal(L1, L8)
    assert np.all(L1[np.triu_indices(600, 1)] == 0.0)


def test_empty():
    L, f = oracle.chol(np.zeros((0, 0)))
    assert L.shape == (0, 0) and f == -1


MUTANTS = {
    "dropped_last_term": ("        double prod = li[p] * lj[p];\n        v = v - prod;",
                          "        if (p + 1 == j) break;\n        double prod = li[p] * lj[p];\n"
                          "        v = v - prod;"),
    "dropped_pivot_term": ("      double prod = lj[p] * lj[p];\n      piv = piv - prod;",
                           "      if (p == 0) continue;\n      double prod = lj[p] * lj[p];\n"
                           "      piv = piv - prod;"),
    "wrong_sign": ("        v = v - prod;", "        v = v + prod;"),
    "no_square_root": ("const double d = sqrt(piv);", "const double d = piv;"),
    "wrong_row": ("double prod = li[p] * lj[p];", "double prod = li[p] * li[p];"),
    "reads_upper": ("for (int64_t j = 0; j <= i; ++j) li[j] = ai[j];",
                    "for (int64_t j = 0; j <= i; ++j) li[j] = A[j * lda + i];"),
    "failure_off_by_one": ("      if (fail) *fail = j;\n      return 0;",
                           "      if (fail) *fail = j + 1;\n      return 0;"),
    "no_division": ("li[j] = v / d;", "li[j] = v;"),
}


def _compile(src, tmp_path):
    c, so = tmp_path / "mut_chol.c", tmp_path / "mut_chol.so"
    c.write_text(src)
    subprocess.run(["gcc", *oracle.CFLAGS, str(c), "-o", str(so), *oracle.LIBS], check=True)
    lib = ctypes.CDLL(str(so))
    i64, dp = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_chol_f64.argtypes = [i64, dp, i64, dp, i64, ctypes.c_int, ctypes.POINTER(i64)]
    lib.oracle_chol_f64.restype = ctypes.c_int

    def chol(A):
        A = np.ascontiguousarray(A, dtype=np.float64)
        n = A.shape[0]
        L = np.zeros_like(A)
        f = ctypes.c_int64(-1)
        lib.oracle_chol_f64(n, A.ctypes.data, n, L.ctypes.data, n, 1, ctypes.byref(f))
        return L, int(f.value)
    return chol


def test_unmodified_source_passes(tmp_path):
    assert _failed_pins(_compile(SRC, tmp_path)) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    assert SRC.count(old) == 1, "mutation anchor must be unique in oracle.c"
    failed = _failed_pins(_compile(SRC.replace(old, new, 1), tmp_path))
    assert failed, f"mutant {name} passed every pin"
