"""Pins for the oracle's Frobenius norms and the two error measures built on
them (relative forward error ||X - Xref||_F / ||Xref||_F and normwise backward
error ||B - L X||_F / (||L||_F ||X||_F), the postcondition B = L X of
Alg. It-Inv-TRSM measured as a defect).  Every parity tolerance in the test
suite goes through these functions, so each is checked against facts that do
not come from the oracle: closed forms (||I_n||_F = sqrt(n), the all-ones
lower triangle gives sqrt(n(n+1)/2), diag(d) gives ||d||_2), exact rational
sums of squares with one correctly rounded square root, numpy's LAPACK-based
norm, and exact power-of-two error ratios.

``failed_norm_pins(mod)`` runs every pin against a module exposing ``fro``,
``fro_lower``, ``rel_fro_err`` and ``backward_err`` and returns the names of
the pins that fail; it is shared by the direct tests and the planted-mistake
tests.  CPU only."""
from decimal import Decimal, getcontext
from fractions import Fraction
import math

import numpy as np

from paper_1612_01855_amd import inputs as gen

NAN = float("nan")


def sqrt_rounded(q: Fraction) -> float:
    """sqrt of an exact non-negative rational, rounded to binary64 (80 decimal
    digits before the final rounding: far more than a double needs)."""
    getcontext().prec = 80
    if q == 0:
        return 0.0
    return float((Decimal(q.numerator) / Decimal(q.denominator)).sqrt())


def exact_sumsq(vals) -> Fraction:
    return sum((Fraction(float(v)) ** 2 for v in vals), Fraction(0))


def _ulps(a: float, b: float) -> float:
    if a == b:
        return 0.0
    if not (math.isfinite(a) and math.isfinite(b)):
        return math.inf
    return abs(a - b) / math.ulp(max(abs(a), abs(b)))


def _with_nan_upper(L):
    L = np.array(L, dtype=np.float64)
    L[np.triu_indices(L.shape[0], 1)] = NAN
    return L


def failed_norm_pins(mod):
    failed = []

    # ||I_n||_F = sqrt(n): one correctly rounded square root of an integer
    for n in (1, 4, 7, 100):
        if mod.fro_lower(_with_nan_upper(gen.identity(n))) != math.sqrt(n):
            failed.append(f"identity_lower_{n}")
        if mod.fro(gen.identity(n)) != math.sqrt(n):
            failed.append(f"identity_dense_{n}")

    # all-ones lower triangle: n(n+1)/2 ones
    for n in (1, 3, 10, 64):
        if mod.fro_lower(_with_nan_upper(gen.ones_lower(n))) != math.sqrt(n * (n + 1) // 2):
            failed.append(f"ones_lower_{n}")

    # diag(d): ||d||_2 from the exact sum of squares
    for n, seed in ((5, 1), (40, 2)):
        L = gen.diagonal(n, seed)
        d = np.diag(L).copy()
        if _ulps(mod.fro_lower(_with_nan_upper(L)), sqrt_rounded(exact_sumsq(d))) > 1:
            failed.append(f"diagonal_{n}")

    # random lower triangles at n <= 8: the exact rational sum of squares of
    # the lower triangle (diagonal included), rounded once
    for n in (2, 5, 8):
        L = gen.rng(10 + n).uniform(-3.0, 3.0, size=(n, n))
        ref = sqrt_rounded(exact_sumsq(L[np.tril_indices(n)]))
        if _ulps(mod.fro_lower(_with_nan_upper(L)), ref) > 1:
            failed.append(f"exact_lower_{n}")

    # dense: exact rational at small sizes, and a row stride wider than the
    # row (the columns past k hold NaN and must not be read)
    for (n, k) in ((3, 4), (7, 2)):
        A = gen.rng(20 + n).normal(size=(n, k))
        if _ulps(mod.fro(A), sqrt_rounded(exact_sumsq(A.ravel()))) > 1:
            failed.append(f"exact_dense_{n}x{k}")
    wide = gen.rng(31).normal(size=(9, 11))
    wide[:, 6:] = NAN
    view = wide[:, :6]
    if _ulps(mod.fro(view), sqrt_rounded(exact_sumsq(view.ravel()))) > 1:
        failed.append("dense_leading_dimension")
    # a lower-triangle view with a wide row stride
    wideL = gen.rng(32).uniform(-1.0, 1.0, size=(6, 10))
    wideL[:, 6:] = NAN
    viewL = wideL[:, :6]
    ref = sqrt_rounded(exact_sumsq(viewL[np.tril_indices(6)]))
    if _ulps(mod.fro_lower(viewL), ref) > 1:
        failed.append("lower_leading_dimension")

    # numpy (LAPACK dnrm2-style scaling) on larger random matrices
    A = gen.rng(40).normal(size=(123, 77))
    if _ulps(mod.fro(A), float(np.linalg.norm(A))) > 8:
        failed.append("numpy_dense")
    L = gen.rng(41).normal(size=(150, 150))
    if _ulps(mod.fro_lower(_with_nan_upper(L)), float(np.linalg.norm(np.tril(L)))) > 8:
        failed.append("numpy_lower")

    # relative error: X = Xref (1 + 2^-20) is exact for small integers, and
    # ||2^-20 Xref|| / ||Xref|| = 2^-20 exactly (powers of two scale exactly)
    Xref = gen.int_rhs(13, 5, 7).astype(np.float64)
    Xref[0, 0] = 3.0
    X = Xref * (1.0 + 2.0 ** -20)
    if mod.rel_fro_err(X, Xref) != 2.0 ** -20:
        failed.append("rel_err_pow2")
    if mod.rel_fro_err(Xref, Xref) != 0.0:
        failed.append("rel_err_zero")
    # the denominator is the reference's norm, not the candidate's
    if mod.rel_fro_err(2.0 * Xref, Xref) != 1.0:
        failed.append("rel_err_denominator")

    # backward error, closed form: L = 2 I (n = 4, NaN above the diagonal),
    # X = all ones, B = L X except one entry off by 1/2:
    # ||R|| = 1/2, ||L|| = 2 sqrt(4) = 4, ||X|| = 4  =>  2^-5
    n = 4
    L = _with_nan_upper(2.0 * np.eye(n))
    X = np.ones((n, n))
    B = 2.0 * np.ones((n, n))
    B[2, 1] += 0.5
    if mod.backward_err(L, X, B) != 2.0 ** -5:
        failed.append("backward_closed_form")
    # backward error against exact rationals: all-ones lower L (n = 3),
    # integer X, B = L X + E with a known defect E
    n, k = 3, 2
    L = _with_nan_upper(gen.ones_lower(n))
    X = np.array([[1.0, -2.0], [3.0, 0.5], [-1.0, 2.0]])
    E = np.array([[0.25, 0.0], [0.0, -0.5], [0.125, 0.0]])
    B = np.tril(np.nan_to_num(L)) @ X + E
    num = sqrt_rounded(exact_sumsq(E.ravel()))
    den_q = exact_sumsq(np.ones(6)) * exact_sumsq(X.ravel())
    ref = float(Fraction(num) / Fraction(sqrt_rounded(den_q)))
    if _ulps(mod.backward_err(L, X, B), ref) > 2:
        failed.append("backward_exact")
    return failed
