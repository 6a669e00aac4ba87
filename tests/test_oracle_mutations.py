"""Planted mistakes in the oracle must be caught by its pins.

Each case copies ``oracle/oracle.c``, plants one plausible mistake (a
transposed operand, a dropped term, a wrong sign, a wrong index, a product
in place of the division), compiles the copy with the same flags on the CPU
and runs the closed-form and brute-force pins against it.  At least one pin
must fail for every mutant, and all of them must pass for the unmodified
source.  CPU only."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_1612_01855_amd import inputs as gen
from lu_piv_pins import failed_lu_piv_pins
from norm_pins import failed_norm_pins

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()

MUTANTS = {
    "transposed_L": ("const double lij = li[j];", "const double lij = L[j * ldl + i];"),
    "dropped_last_term": ("for (int64_t j = 0; j < i; ++j) {\n      const double lij",
                          "for (int64_t j = 0; j + 1 < i; ++j) {\n      const double lij"),
    "dropped_first_term": ("for (int64_t j = 0; j < i; ++j) {\n      const double lij",
                           "for (int64_t j = 1; j < i; ++j) {\n      const double lij"),
    "wrong_sign": ("xi[c] = xi[c] - prod;", "xi[c] = xi[c] + prod;"),
    "wrong_x_row": ("const double* xj = X + j * ldx;", "const double* xj = X + i * ldx;"),
    "multiply_not_divide": ("xi[c] = xi[c] / d;", "xi[c] = xi[c] * d;"),
    "wrong_diagonal": ("const double d = li[i];", "const double d = L[i * ldl + (i ? i - 1 : 0)];"),
    "rhs_wrong_column": ("xi[c] = bi[c];", "xi[c] = bi[c0];"),
}


# Planted mistakes in the Frobenius norms every tolerance goes through.
NORM_MUTANTS = {
    "lower_no_sqrt": ("for (int it = 0; it < 3; ++it) r = 0.5Q * (r + s / r);\n  return (double)r;\n}\n\ndouble oracle_fro_dense",
                      "for (int it = 0; it < 3; ++it) r = 0.5Q * (r + s / r);\n  return (double)s;\n}\n\ndouble oracle_fro_dense"),
    "dense_no_sqrt": ("for (int it = 0; it < 3; ++it) r = 0.5Q * (r + s / r);\n  return (double)r;\n}\n\n/* Cholesky",
                      "for (int it = 0; it < 3; ++it) r = 0.5Q * (r + s / r);\n  return (double)s;\n}\n\n/* Cholesky"),
    "lower_drops_diagonal": ("for (int64_t j = 0; j <= i; ++j) {\n      __float128 v = (__float128)L[i * ldl + j];",
                             "for (int64_t j = 0; j < i; ++j) {\n      __float128 v = (__float128)L[i * ldl + j];"),
    "lower_reads_upper": ("__float128 v = (__float128)L[i * ldl + j];",
                          "__float128 v = (__float128)L[j * ldl + i];"),
    "lower_wrong_leading_dim": ("__float128 v = (__float128)L[i * ldl + j];",
                                "__float128 v = (__float128)L[i * n + j];"),
    "dense_wrong_leading_dim": ("__float128 v = (__float128)A[i * lda + c];",
                                "__float128 v = (__float128)A[i * k + c];"),
    "dense_drops_last_column": ("for (int64_t c = 0; c < k; ++c) {\n      __float128 v = (__float128)A[i * lda + c];",
                                "for (int64_t c = 0; c + 1 < k; ++c) {\n      __float128 v = (__float128)A[i * lda + c];"),
    "lower_sum_not_squared": ("      s += v * v;\n    }\n  /* square root",
                              "      s += v < 0 ? -v : v;\n    }\n  /* square root"),
}


# Planted mistakes in LU with partial pivoting.
LU_PIV_MUTANTS = {
    "last_largest_on_ties": ("if (v > best) {\n        best = v;\n        p = i;",
                             "if (v >= best) {\n        best = v;\n        p = i;"),
    "signed_not_magnitude": ("const double v = fabs(LU[i * ldu + j]);",
                             "const double v = LU[i * ldu + j];"),
    "search_skips_a_row": ("for (int64_t i = j + 1; i < n; ++i) {\n      const double v = fabs",
                           "for (int64_t i = j + 2; i < n; ++i) {\n      const double v = fabs"),
    "exchange_skips_L_part": ("for (int64_t c = 0; c < n; ++c) {\n        const double t = rj[c];",
                              "for (int64_t c = j; c < n; ++c) {\n        const double t = rj[c];"),
    "no_exchange": ("    if (p != j) {\n      double* rj", "    if (0) {\n      double* rj"),
    "ipiv_records_step": ("    ipiv[j] = p;", "    ipiv[j] = j;"),
    "multiplier_multiplies": ("const double l = ri[j] / piv;", "const double l = ri[j] * piv;"),
    "update_skips_last_column": ("for (int64_t c = j + 1; c < n; ++c) {\n        const double term = l * uj[c];",
                                 "for (int64_t c = j + 1; c + 1 < n; ++c) {\n        const double term = l * uj[c];"),
    "update_wrong_sign": ("ri[c] = ri[c] - term;", "ri[c] = ri[c] + term;"),
}


def _compile(src: str, tmp_path) -> ctypes.CDLL:
    c = tmp_path / "mut.c"
    so = tmp_path / "mut.so"
    c.write_text(src)
    subprocess.run(["gcc", *oracle.CFLAGS, str(c), "-o", str(so), *oracle.LIBS], check=True)
    lib = ctypes.CDLL(str(so))
    i64, dp = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_trsm_f64.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, ctypes.c_int]
    lib.oracle_trsm_f64.restype = ctypes.c_int
    return lib


def _solver(lib):
    def trsm(L, B):
        L = np.ascontiguousarray(L, dtype=np.float64)
        B = np.ascontiguousarray(B, dtype=np.float64)
        n, k = B.shape
        X = np.empty_like(B)
        lib.oracle_trsm_f64(n, k, L.ctypes.data, n, B.ctypes.data, k, X.ctypes.data, k, 1)
        return X
    return trsm


def _failed_pins(trsm):
    failed = []
    n, k = 12, 3
    L = gen.identity(n)
    L[np.triu_indices(n, 1)] = np.nan
    B = gen.rhs(n, k, 1)
    if not np.array_equal(trsm(L, B), B):
        failed.append("identity")
    L = gen.diagonal(n, 2)
    d = np.diag(L).copy()
    L[np.triu_indices(n, 1)] = np.nan
    if not np.array_equal(trsm(L, B), B / d[:, None]):
        failed.append("diagonal")
    L = gen.bidiagonal_minus_one(n)
    L[np.triu_indices(n, 1)] = np.nan
    if not np.array_equal(trsm(L, B), np.cumsum(B, axis=0)):
        failed.append("bidiagonal")
    L = gen.ones_lower(n)
    L[np.triu_indices(n, 1)] = np.nan
    Bi = gen.int_rhs(n, k, 5)
    expect = Bi.copy()
    expect[1:] -= Bi[:-1]
    if not np.array_equal(trsm(L, Bi), expect):
        failed.append("ones_lower")
    L, B = gen.easy_system(6, 2, 0)
    X = trsm(L, B)
    if not np.all(np.isfinite(X)):
        failed.append("brute_force")
    else:
        Xq = exact.solve(L, B)
        bound = exact.substitution_bound(L, X, n_ops=7)
        if any(abs(exact.Fraction(float(X[i, c])) - Xq[i][c]) > bound[i][c]
               for i in range(6) for c in range(2)):
            failed.append("brute_force")
    return failed


def test_unmodified_source_passes_all_pins(tmp_path):
    assert _failed_pins(_solver(_compile(SRC, tmp_path))) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    assert SRC.count(old) >= 1, "mutation anchor not found in oracle.c"
    mutated = SRC.replace(old, new, 1)
    failed = _failed_pins(_solver(_compile(mutated, tmp_path)))
    assert failed, f"mutant {name} passed every pin"


def test_unmodified_source_passes_norm_pins(tmp_path, monkeypatch):
    monkeypatch.setattr(oracle, "_lib", oracle.bind(_compile(SRC, tmp_path)))
    assert failed_norm_pins(oracle) == []


@pytest.mark.parametrize("name", sorted(NORM_MUTANTS))
def test_norm_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = NORM_MUTANTS[name]
    assert SRC.count(old) == 1, "mutation anchor not found once in oracle.c"
    lib = oracle.bind(_compile(SRC.replace(old, new, 1), tmp_path))
    monkeypatch.setattr(oracle, "_lib", lib)
    failed = failed_norm_pins(oracle)
    assert failed, f"norm mutant {name} passed every pin"


def test_unmodified_source_passes_lu_piv_pins(tmp_path, monkeypatch):
    monkeypatch.setattr(oracle, "_lib", oracle.bind(_compile(SRC, tmp_path)))
    assert failed_lu_piv_pins(oracle.lu_piv) == []


@pytest.mark.parametrize("name", sorted(LU_PIV_MUTANTS))
def test_lu_piv_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = LU_PIV_MUTANTS[name]
    assert SRC.count(old) == 1, "mutation anchor not found once in oracle.c"
    lib = oracle.bind(_compile(SRC.replace(old, new, 1), tmp_path))
    monkeypatch.setattr(oracle, "_lib", lib)
    failed = failed_lu_piv_pins(oracle.lu_piv)
    assert failed, f"LU mutant {name} passed every pin"
