"""CPU oracle for the triangular solve L X = B -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library (``include/trsm.h``,
``paper_1612_01855_amd``) never imports, links or calls it, and the two share
no code: the only thing both sides use is the seeded input generator module
``paper_1612_01855_amd.inputs``, which holds none of the method's arithmetic.

What it computes (all in IEEE binary64 unless stated):

* ``trsm(L, B)`` -- X = L^{-1} B by plain forward substitution, the definition
  of the problem in Sec. I (L lower triangular n x n, B and X dense n x k).
  The paper's method (Alg. It-Inv-TRSM, Sec. VI) ensures B = L X, so every GPU
  variant (any n0, right- or left-looking, any precision that is refined back
  to binary64) must reach this X up to rounding.
* ``diag_block_inverses(L, n0)`` -- the inverse of every n0 x n0 diagonal
  block S_i = i*n0 : (i+1)*n0 (Alg. Diagonal-Inverter, whose postcondition is
  that each inverted block times the original block is the identity), computed
  by forward substitution on identity columns; the last block is ragged when
  n0 does not divide n.
* ``residual(L, X, B)`` -- B - L X summed plainly (the postcondition B = L X
  written as a defect).
* ``trsm_q(L, B)`` -- the same substitution in binary128, rounded once.
* ``trsm_t(L, B)`` -- X = L^{-T} B by backward substitution (the transposed
  problem, the second half of a solve with A = L L^T).
* ``chol(A)`` -- the Cholesky factor A = L L^T of a symmetric positive
  definite A by its column-by-column definition (the factorization whose
  panel step is a triangular solve, named in the abstract and Sec. I).
* ``lu_nopiv(A)`` -- LU factors A = L U without row exchanges by Doolittle's
  definition (the other factorization named there, in its no-pivoting form).
* ``oracle.exact`` -- exact rational arithmetic (Gauss-Jordan on Q) for
  brute-force pins at tiny n.

The C source ``oracle.c`` is compiled with ``-O2 -ffp-contract=off
-fno-fast-math`` so that every product is rounded before it is subtracted and
the division is a true division.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_BUILD_DIR = os.path.join(_HERE, "_build")
_SO = os.path.join(_BUILD_DIR, "liboracle.so")

_lib = None
_lock = threading.Lock()

CFLAGS = ["-O2", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
          "-fno-fast-math", "-ffp-contract=off", "-std=gnu11"]
LIBS = ["-lquadmath", "-lm"]


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``_build/liboracle.so`` with gcc."""
    os.makedirs(_BUILD_DIR, exist_ok=True)
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", *CFLAGS, _SRC, "-o", tmp, *LIBS]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_SO):
            build(force=False)
        _lib = bind(ctypes.CDLL(_SO))
        return _lib


def bind(lib):
    """Declare the argument and result types of the library's functions (also
    used on copies compiled from planted-mistake sources in the tests)."""
    i64, dp, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
    for name in ("oracle_trsm_f64", "oracle_trsm_q", "oracle_trsm_t_f64"):
        f = getattr(lib, name)
        f.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, ci]
        f.restype = ci
    lib.oracle_residual_f64.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, dp, i64, ci]
    lib.oracle_residual_f64.restype = ci
    lib.oracle_fro_lower.argtypes = [i64, dp, i64]
    lib.oracle_fro_lower.restype = ctypes.c_double
    lib.oracle_fro_dense.argtypes = [i64, i64, dp, i64]
    lib.oracle_fro_dense.restype = ctypes.c_double
    lib.oracle_chol_f64.argtypes = [i64, dp, i64, dp, i64, ci, ctypes.POINTER(i64)]
    lib.oracle_chol_f64.restype = ci
    lib.oracle_lu_nopiv_f64.argtypes = [i64, dp, i64, dp, i64, ci, ctypes.POINTER(i64)]
    lib.oracle_lu_nopiv_f64.restype = ci
    lib.oracle_lu_piv_f64.argtypes = [i64, dp, i64, dp, i64, ci, dp, ctypes.POINTER(i64)]
    lib.oracle_lu_piv_f64.restype = ci
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ci
    return lib


def _rows(a: np.ndarray) -> np.ndarray:
    """Return a float64 2-D array whose rows are unit-stride (row-major)."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim != 2:
        raise ValueError("expected a 2-D array")
    if a.strides[1] != 8 or a.strides[0] < 8 * max(a.shape[1], 1) or a.strides[0] % 8:
        a = np.ascontiguousarray(a)
    return a


def _ld(a: np.ndarray) -> int:
    return max(a.strides[0] // 8, a.shape[1], 1)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def trsm(L, B, nthreads: int = 0) -> np.ndarray:
    """X = L^{-1} B by forward substitution (Sec. I).  Reads only the lower
    triangle of ``L`` (diagonal included)."""
    lib = _load()
    L, B = _rows(L), _rows(B)
    n, k = B.shape
    if L.shape[0] != n or L.shape[1] < n:
        raise ValueError("L must be n x n with n = B.shape[0]")
    X = np.empty((n, k), dtype=np.float64)
    rc = lib.oracle_trsm_f64(n, k, L.ctypes.data, _ld(L), B.ctypes.data, _ld(B),
                             X.ctypes.data, max(k, 1), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_trsm_f64 rejected the sizes")
    return X


def trsm_t(L, B, nthreads: int = 0) -> np.ndarray:
    """X = L^{-T} B by backward substitution (the transposed problem L^T X =
    B).  Reads only the lower triangle of ``L`` (diagonal included)."""
    lib = _load()
    L, B = _rows(L), _rows(B)
    n, k = B.shape
    if L.shape[0] != n or L.shape[1] < n:
        raise ValueError("L must be n x n with n = B.shape[0]")
    X = np.empty((n, k), dtype=np.float64)
    rc = lib.oracle_trsm_t_f64(n, k, L.ctypes.data, _ld(L), B.ctypes.data, _ld(B),
                               X.ctypes.data, max(k, 1), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_trsm_t_f64 rejected the sizes")
    return X


def trsm_q(L, B, nthreads: int = 0) -> np.ndarray:
    """Forward substitution in binary128, result rounded once to binary64."""
    lib = _load()
    L, B = _rows(L), _rows(B)
    n, k = B.shape
    X = np.empty((n, k), dtype=np.float64)
    rc = lib.oracle_trsm_q(n, k, L.ctypes.data, _ld(L), B.ctypes.data, _ld(B),
                           X.ctypes.data, max(k, 1), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_trsm_q rejected the sizes")
    return X


def residual(L, X, B, nthreads: int = 0) -> np.ndarray:
    """R = B - L X with the lower triangle of L, summed plainly."""
    lib = _load()
    L, X, B = _rows(L), _rows(X), _rows(B)
    n, k = B.shape
    R = np.empty((n, k), dtype=np.float64)
    rc = lib.oracle_residual_f64(n, k, L.ctypes.data, _ld(L), X.ctypes.data, _ld(X),
                                 B.ctypes.data, _ld(B), R.ctypes.data, max(k, 1),
                                 int(nthreads))
    if rc != 0:
        raise ValueError("oracle_residual_f64 rejected the sizes")
    return R


def fro_lower(L) -> float:
    """Frobenius norm of the lower triangle of L (diagonal included)."""
    L = _rows(L)
    return float(_load().oracle_fro_lower(L.shape[0], L.ctypes.data, _ld(L)))


def fro(A) -> float:
    """Frobenius norm of a dense matrix."""
    A = _rows(A)
    return float(_load().oracle_fro_dense(A.shape[0], A.shape[1], A.ctypes.data, _ld(A)))


def inv_lower(L) -> np.ndarray:
    """L^{-1} by forward substitution on the columns of the identity."""
    n = np.asarray(L).shape[0]
    return trsm(L, np.eye(n))


def diag_block_inverses(L, n0: int) -> list:
    """Inverse of every diagonal block L(S_i, S_i), S_i = i*n0 : min((i+1)*n0, n)
    (Alg. Diagonal-Inverter: each inverted block times its block is the
    identity).  Returns a list of square arrays; the last one is ragged when n0
    does not divide n."""
    L = _rows(L)
    n = L.shape[0]
    out = []
    for s in range(0, n, n0):
        e = min(s + n0, n)
        out.append(inv_lower(L[s:e, s:e]))
    return out


def chol(A, nthreads: int = 0):
    """Cholesky factor of a symmetric positive definite A (lower triangle
    read): returns (L, fail) with L lower triangular, zeros above the
    diagonal, A = L L^T, and fail = -1, or the first column whose pivot is not
    positive (L's columns from there on are then unspecified)."""
    lib = _load()
    A = _rows(A)
    n = A.shape[0]
    if A.shape[1] < n:
        raise ValueError("A must be n x n")
    L = np.empty((n, n), dtype=np.float64)
    fail = ctypes.c_int64(-1)
    rc = lib.oracle_chol_f64(n, A.ctypes.data, _ld(A), L.ctypes.data, max(n, 1),
                             int(nthreads), ctypes.byref(fail))
    if rc != 0:
        raise ValueError("oracle_chol_f64 rejected the sizes")
    return L, int(fail.value)


def lu_nopiv(A, nthreads: int = 0):
    """LU factors without pivoting, A = L U (Doolittle): returns (L, U, fail)
    with L unit lower triangular, U upper triangular, and fail = -1, or the
    first step whose pivot is zero or not finite (the factors are then
    unspecified from there on)."""
    lib = _load()
    A = _rows(A)
    n = A.shape[0]
    if A.shape[1] < n:
        raise ValueError("A must be n x n")
    LU = np.empty((n, n), dtype=np.float64)
    fail = ctypes.c_int64(-1)
    rc = lib.oracle_lu_nopiv_f64(n, A.ctypes.data, _ld(A), LU.ctypes.data, max(n, 1),
                                 int(nthreads), ctypes.byref(fail))
    if rc != 0:
        raise ValueError("oracle_lu_nopiv_f64 rejected the sizes")
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    return L, U, int(fail.value)


def lu_piv(A, nthreads: int = 0):
    """LU factors with partial pivoting, P A = L U (Gaussian elimination with
    row exchanges, LAPACK dgetf2's order): returns (L, U, ipiv, fail) with L
    unit lower triangular, U upper triangular, ipiv[j] (0-based, >= j) the row
    exchanged with row j at step j, and fail = -1 or the first step whose
    pivot is zero."""
    lib = _load()
    A = _rows(A)
    n = A.shape[0]
    if A.shape[1] < n:
        raise ValueError("A must be n x n")
    LU = np.empty((n, n), dtype=np.float64)
    ipiv = np.empty(max(n, 1), dtype=np.int64)
    fail = ctypes.c_int64(-1)
    rc = lib.oracle_lu_piv_f64(n, A.ctypes.data, _ld(A), LU.ctypes.data, max(n, 1),
                               int(nthreads), ipiv.ctypes.data, ctypes.byref(fail))
    if rc != 0:
        raise ValueError("oracle_lu_piv_f64 rejected the sizes")
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    return L, U, ipiv[:n].copy(), int(fail.value)


def perm_from_ipiv(ipiv) -> np.ndarray:
    """The row order p with (P A) = A[p] for the exchanges "swap rows j and
    ipiv[j]", j ascending."""
    p = np.arange(len(ipiv))
    for j, q in enumerate(ipiv):
        q = int(q)
        if q != j:
            p[j], p[q] = p[q], p[j]
    return p


def rel_fro_err(X, Xref) -> float:
    """||X - Xref||_F / ||Xref||_F (relative normwise error, Frobenius)."""
    X = np.asarray(X, dtype=np.float64)
    Xref = np.asarray(Xref, dtype=np.float64)
    den = fro(Xref)
    num = fro(X - Xref)
    if den == 0.0:
        return num
    return num / den


def backward_err(L, X, B) -> float:
    """||B - L X||_F / (||L||_F ||X||_F) over the lower triangle of L."""
    R = residual(L, X, B)
    den = fro_lower(L) * fro(X)
    return fro(R) / den if den else fro(R)
