"""Pins of the transposed oracle, X = L^{-T} B by backward substitution (the
problem L^T X = B, the second half of a solve with A = L L^T), and planted
mistakes in it that the pins must catch.  CPU only.

Closed forms: for L = I, diag(d); for the unit lower bidiagonal L with -1 on
the subdiagonal, L^T is unit upper bidiagonal with -1 above the diagonal and
(L^T)^{-1} is the all-ones upper triangle, so X is the suffix sum of B; for
the all-ones lower triangle, (L^T)^{-1} has 1 on the diagonal and -1 above
it, so X_i = B_i - B_{i+1}.  Brute force: exact rational solutions at n <= 8
within the substitution bound.  A different algorithm: reversing the order of
rows and columns turns L^T into a lower-triangular matrix, which the forward
oracle solves."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_1612_01855_amd import inputs as gen

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()


def _nan_upper(L):
    L = np.array(L, dtype=np.float64)
    L[np.triu_indices(L.shape[0], 1)] = np.nan
    return L


def _flip_solve(L, B):
    """X from the forward oracle on the reversed problem: P L^T P (P X) = P B."""
    M = np.ascontiguousarray(L.T[::-1, ::-1])
    return oracle.trsm(M, np.ascontiguousarray(B[::-1]))[::-1]


def _failed_pins(trsm_t):
    failed = []
    n, k = 12, 3
    B = gen.rhs(n, k, 1)
    if not np.array_equal(trsm_t(_nan_upper(gen.identity(n)), B), B):
        failed.append("identity")
    Ld = gen.diagonal(n, 2)
    d = np.diag(Ld).copy()
    if not np.array_equal(trsm_t(_nan_upper(Ld), B), B / d[:, None]):
        failed.append("diagonal")
    Bi = gen.int_rhs(n, k, 5)
    if not np.array_equal(trsm_t(_nan_upper(gen.bidiagonal_minus_one(n)), Bi),
                          np.cumsum(Bi[::-1], axis=0)[::-1]):
        failed.append("bidiagonal")
    expect = Bi.copy()
    expect[:-1] -= Bi[1:]
    if not np.array_equal(trsm_t(_nan_upper(gen.ones_lower(n)), Bi), expect):
        failed.append("ones_lower")
    L, B6 = gen.easy_system(6, 2, 0)
    X = trsm_t(_nan_upper(L), B6)
    if not np.all(np.isfinite(X)):
        failed.append("brute_force")
    else:
        M = L.T[::-1, ::-1]
        Xq = exact.solve(M, B6[::-1])
        bound = exact.substitution_bound(M, X[::-1], n_ops=7)
        if any(abs(exact.Fraction(float(X[5 - i, c])) - Xq[i][c]) > bound[i][c]
               for i in range(6) for c in range(2)):
            failed.append("brute_force")
    return failed


def test_oracle_passes_its_pins():
    assert _failed_pins(oracle.trsm_t) == []


@pytest.mark.parametrize("n,k", [(1, 1), (40, 7), (300, 70)])
def test_reversed_problem_agrees(n, k):
    L, B = gen.easy_system(n, k, n + 3)
    X = oracle.trsm_t(_nan_upper(L), B)
    assert oracle.rel_fro_err(X, _flip_solve(L, B)) <= 1e-14


@pytest.mark.parametrize("gen_name,n,k", [("easy", 500, 9), ("chol", 400, 5)])
def test_residual_invariant(gen_name, n, k):
    L = gen.easy_lower(n, 4) if gen_name == "easy" else gen.chol_lower(n, 4)
    B = gen.rhs(n, k, 4)
    X = oracle.trsm_t(L, B)
    R = B - np.tril(L).T @ X
    assert oracle.fro(R) <= 1e-14 * oracle.fro_lower(L) * oracle.fro(X)


def test_column_split_and_in_place_are_bitwise():
    L, B = gen.easy_system(200, 150, 9, upper=np.nan)
    X1 = oracle.trsm_t(L, B, nthreads=1)
    X4 = oracle.trsm_t(L, B, nthreads=4)
    assert np.array_equal(X1, X4)
    Xa = np.concatenate([oracle.trsm_t(L, B[:, :64]), oracle.trsm_t(L, B[:, 64:])], axis=1)
    assert np.array_equal(X1, Xa)


def test_empty_sizes():
    assert oracle.trsm_t(np.zeros((0, 0)), np.zeros((0, 3))).shape == (0, 3)
    assert oracle.trsm_t(np.eye(4), np.zeros((4, 0))).shape == (4, 0)


MUTANTS = {
    "untransposed_L": ("const double lji = L[j * ldl + i];", "const double lji = L[i * ldl + j];"),
    "dropped_last_term": ("for (int64_t j = i + 1; j < n; ++j) {",
                          "for (int64_t j = i + 1; j + 1 < n; ++j) {"),
    "dropped_first_term": ("for (int64_t j = i + 1; j < n; ++j) {",
                           "for (int64_t j = i + 2; j < n; ++j) {"),
    "forward_order": ("for (int64_t i = n - 1; i >= 0; --i) {", "for (int64_t i = 0; i < n; ++i) {"),
    "wrong_sign": ("        double prod = lji * xj[c];\n        xi[c] = xi[c] - prod;",
                   "        double prod = lji * xj[c];\n        xi[c] = xi[c] + prod;"),
    "wrong_diagonal": ("const double d = L[i * ldl + i];",
                       "const double d = L[i * ldl + (i ? i - 1 : 0)];"),
}


def _compile(src, tmp_path):
    c, so = tmp_path / "mut_t.c", tmp_path / "mut_t.so"
    c.write_text(src)
    subprocess.run(["gcc", *oracle.CFLAGS, str(c), "-o", str(so), *oracle.LIBS], check=True)
    lib = ctypes.CDLL(str(so))
    i64, dp = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_trsm_t_f64.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, ctypes.c_int]
    lib.oracle_trsm_t_f64.restype = ctypes.c_int

    def trsm_t(L, B):
        L = np.ascontiguousarray(L, dtype=np.float64)
        B = np.ascontiguousarray(B, dtype=np.float64)
        n, k = B.shape
        X = np.zeros_like(B)
        lib.oracle_trsm_t_f64(n, k, L.ctypes.data, n, B.ctypes.data, k, X.ctypes.data, k, 1)
        return X
    return trsm_t


def test_unmodified_source_passes(tmp_path):
    assert _failed_pins(_compile(SRC, tmp_path)) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    assert SRC.count(old) == 1, "mutation anchor must be unique in oracle.c"
    failed = _failed_pins(_compile(SRC.replace(old, new, 1), tmp_path))
    assert failed, f"mutant {name} passed every pin"
