"""Pins of the LU oracle without row exchanges, A = L U by Doolittle's
definition (L unit lower, U upper), and planted mistakes in it that the pins
must catch.  CPU only.

Exact pins: for an integer unit-lower L and an integer upper U whose diagonal
holds +-1, +-2 or +-4, A = L U is an integer matrix, every intermediate of the
definition is an integer (or an exact division by a power of two), so the
oracle must return L and U bit for bit; the identity and diagonal matrices.
A library routine: LAPACK's partially pivoted LU (scipy) on strictly column
diagonally dominant matrices, where partial pivoting exchanges no row.  A
different factorization: for symmetric positive definite A, L U = C C^T
(Cholesky oracle) gives L = C diag(1/c_jj) and U = diag(c_jj) C^T.
Invariants: the componentwise backward error bound |A - L U| <= gamma_n |L||U|
and the index of the first zero pivot."""
import ctypes
import os
import subprocess

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_1612_01855_amd import inputs as gen

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
U64 = 2.0 ** -53


def _int_pair(n, seed):
    L0 = gen.int_unit_lower_small(n, seed)
    U0 = gen.int_upper_pow2(n, seed + 1)
    A = (L0.astype(np.int64) @ U0.astype(np.int64)).astype(np.float64)
    return L0, U0, A


def _failed_pins(lu):
    failed = []
    L0, U0, A = _int_pair(24, 3)
    L, U, f = lu(A)
    if f != -1 or not (np.array_equal(L, L0) and np.array_equal(U, U0)):
        failed.append("integer_factors")
    d = gen.rng(5).uniform(0.5, 4.0, size=9)
    L, U, f = lu(np.diag(d))
    if f != -1 or not (np.array_equal(L, np.eye(9)) and np.array_equal(U, np.diag(d))):
        failed.append("diagonal")
    A = gen.diag_dominant(60, 7)
    L, U, f = lu(A)
    P, Ls, Us = scipy.linalg.lu(A)
    if (f != -1 or not np.array_equal(P, np.eye(60))
            or oracle.rel_fro_err(L, Ls) > 1e-14 or oracle.rel_fro_err(U, Us) > 1e-14):
        failed.append("lapack")
    L0, U0, A = _int_pair(12, 8)
    U0z = U0.copy()
    U0z[7, 7] = 0.0
    Az = (L0.astype(np.int64) @ U0z.astype(np.int64)).astype(np.float64)
    _, U, f = lu(Az)
    if f != 7 or not np.array_equal(U[:7], U0z[:7]):
        failed.append("failure_index")
    return failed


def test_oracle_passes_its_pins():
    assert _failed_pins(oracle.lu_nopiv) == []


@pytest.mark.parametrize("n", [1, 33, 250])
def test_agrees_with_lapack_on_diagonally_dominant(n):
    A = gen.diag_dominant(n, n)
    L, U, f = oracle.lu_nopiv(A)
    P, Ls, Us = scipy.linalg.lu(A)
    assert f == -1 and np.array_equal(P, np.eye(n))
    assert oracle.rel_fro_err(L, Ls) <= 1e-14 and oracle.rel_fro_err(U, Us) <= 1e-14


def test_agrees_with_cholesky_on_spd():
    A = gen.spd(200, 3)
    L, U, f = oracle.lu_nopiv(A)
    C, g = oracle.chol(A)
    assert f == -1 and g == -1
    d = np.diag(C)
    assert oracle.rel_fro_err(L, C / d[None, :]) <= 1e-14
    assert oracle.rel_fro_err(U, d[:, None] * C.T) <= 1e-14


@pytest.mark.parametrize("n", [300, 64])
def test_backward_error_bound(n):
    A = gen.diag_dominant(n, 11)
    L, U, f = oracle.lu_nopiv(A)
    gamma = n * U64 / (1 - n * U64)
    assert f == -1
    assert np.all(np.abs(A - L @ U) <= gamma * (np.abs(L) @ np.abs(U)))


def test_threads_are_bitwise():
    A = gen.diag_dominant(600, 4)
    L1, U1, _ = oracle.lu_nopiv(A, nthreads=1)
    L8, U8, _ = oracle.lu_nopiv(A, nthreads=8)
    assert np.array_equal(L1, L8) and np.array_equal(U1, U8)


def test_empty_and_nan_pivot():
    L, U, f = oracle.lu_nopiv(np.zeros((0, 0)))
    assert L.shape == (0, 0) and f == -1
    A = gen.diag_dominant(10, 2)
    A[0, 0] = np.nan
    assert oracle.lu_nopiv(A)[2] == 0


MUTANTS = {
    "u_dropped_last_term": ("        double term = uj[p] * LU[p * ldu + c];\n        acc = acc - term;",
                            "        if (p + 1 == j) break;\n        double term = uj[p] * LU[p * ldu + c];\n"
                            "        acc = acc - term;"),
    "l_dropped_last_term": ("        double term = li[p] * LU[p * ldu + j];\n        acc = acc - term;",
                            "        if (p + 1 == j) break;\n        double term = li[p] * LU[p * ldu + j];\n"
                            "        acc = acc - term;"),
    "u_wrong_index": ("double term = uj[p] * LU[p * ldu + c];", "double term = uj[p] * LU[c * ldu + p];"),
    "l_wrong_index": ("double term = li[p] * LU[p * ldu + j];", "double term = li[p] * LU[j * ldu + p];"),
    "wrong_sign": ("      li[j] = acc / ujj;", "      li[j] = -acc / ujj;"),
    "no_division": ("      li[j] = acc / ujj;", "      li[j] = acc;"),
    "failure_off_by_one": ("      if (fail != NULL) *fail = j;", "      if (fail != NULL) *fail = j + 1;"),
    "u_skips_diagonal": ("    for (int64_t c = j; c < n; ++c) {\n      double acc = uj[c];",
                         "    for (int64_t c = j + 1; c < n; ++c) {\n      double acc = uj[c];"),
}


def _compile(src, tmp_path):
    c, so = tmp_path / "mut_lu.c", tmp_path / "mut_lu.so"
    c.write_text(src)
    subprocess.run(["gcc", *oracle.CFLAGS, str(c), "-o", str(so), *oracle.LIBS], check=True)
    lib = ctypes.CDLL(str(so))
    i64, dp = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_lu_nopiv_f64.argtypes = [i64, dp, i64, dp, i64, ctypes.c_int, ctypes.POINTER(i64)]
    lib.oracle_lu_nopiv_f64.restype = ctypes.c_int

    def lu(A):
        A = np.ascontiguousarray(A, dtype=np.float64)
        n = A.shape[0]
        LU = np.zeros_like(A)
        f = ctypes.c_int64(-1)
        lib.oracle_lu_nopiv_f64(n, A.ctypes.data, n, LU.ctypes.data, n, 1, ctypes.byref(f))
        return np.tril(LU, -1) + np.eye(n), np.triu(LU), int(f.value)
    return lu


def test_unmodified_source_passes(tmp_path):
    assert _failed_pins(_compile(SRC, tmp_path)) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    assert SRC.count(old) == 1, "mutation anchor must be unique in oracle.c"
    failed = _failed_pins(_compile(SRC.replace(old, new, 1), tmp_path))
    assert failed, f"mutant {name} passed every pin"
