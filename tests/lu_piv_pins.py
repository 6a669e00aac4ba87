"""Pins for the oracle's LU factorization with partial pivoting, P A = L U
(Gaussian elimination with row exchanges: the first row with the largest
pivot magnitude, LAPACK dgetf2's order).  Each pin checks the oracle against
something that does not come from it: scaled permutation matrices (L = I and
U diagonal, exactly), small cases worked by hand in binary64, ties that the
first-largest rule must break towards the upper row, exact rational
elimination on small integer matrices, LAPACK's dgetrf through
scipy.linalg.lu_factor, the invariants |l_ij| <= 1 and P A = L U to rounding,
and the first zero pivot of singular matrices.

``failed_lu_piv_pins(lu_piv)`` runs every pin against a function with the
signature of ``oracle.lu_piv`` and returns the names of the pins that fail;
it is shared by the direct tests and the planted-mistake tests.  CPU only."""
from fractions import Fraction

import numpy as np

import oracle
from paper_1612_01855_amd import inputs as gen

U64 = 2.0 ** -53


def exact_gepp(A):
    """Gaussian elimination with partial pivoting in exact rationals (first
    largest magnitude on ties).  Returns (L, U, ipiv, tie) with tie True when
    some step had two candidates of equal magnitude after step 0."""
    n = len(A)
    M = [[Fraction(int(v)) for v in row] for row in A]
    ipiv = []
    tie = False
    for j in range(n):
        mags = [abs(M[i][j]) for i in range(j, n)]
        best = max(mags)
        p = j + mags.index(best)
        if j > 0 and best != 0 and mags.count(best) > 1:
            tie = True
        ipiv.append(p)
        M[j], M[p] = M[p], M[j]
        if M[j][j] == 0:
            continue
        for i in range(j + 1, n):
            l = M[i][j] / M[j][j]
            M[i][j] = l
            for c in range(j + 1, n):
                M[i][c] -= l * M[j][c]
    L = [[(M[i][c] if c < i else Fraction(int(c == i))) for c in range(n)] for i in range(n)]
    U = [[(M[i][c] if c >= i else Fraction(0)) for c in range(n)] for i in range(n)]
    return L, U, ipiv, tie


def _close(x: float, q: Fraction, scale: float, rel: float) -> bool:
    return abs(Fraction(float(x)) - q) <= Fraction(rel) * Fraction(scale)


def failed_lu_piv_pins(lu_piv):
    failed = []

    # scaled permutation matrices: every step finds exactly one nonzero
    g = gen.rng(3)
    for n in (1, 7, 16):
        perm = g.permutation(n)
        A = np.zeros((n, n))
        scales = 2.0 ** g.integers(-3, 4, size=n)
        A[perm, np.arange(n)] = scales
        L, U, ipiv, fail = lu_piv(A)
        order = list(range(n))
        exp = []
        for j in range(n):
            p = order.index(int(perm[j]), j)
            exp.append(p)
            order[j], order[p] = order[p], order[j]
        if (fail != -1 or list(ipiv) != exp or not np.array_equal(L, np.eye(n))
                or not np.array_equal(U, np.diag(scales))):
            failed.append("permutation")
            break

    # 2 x 2 by hand: the second row pivots; l = 1/3, u_11 = 2 - l 4 in binary64
    L, U, ipiv, fail = lu_piv(np.array([[1.0, 2.0], [3.0, 4.0]]))
    l = 1.0 / 3.0
    if (list(ipiv) != [1, 1] or fail != -1 or L[1, 0] != l
            or not np.array_equal(U, np.array([[3.0, 4.0], [0.0, 2.0 - l * 4.0]]))):
        failed.append("hand_2x2")

    # ties go to the upper row, at the first step and at a later one
    L, U, ipiv, _ = lu_piv(np.array([[1.0, 5.0], [-1.0, 2.0]]))
    if (list(ipiv) != [0, 1] or L[1, 0] != -1.0
            or not np.array_equal(U, np.array([[1.0, 5.0], [0.0, 7.0]]))):
        failed.append("tie_first_step")
    L, U, ipiv, _ = lu_piv(np.array([[4.0, 0.0, 0.0], [0.0, 1.0, 3.0], [0.0, -1.0, 5.0]]))
    if list(ipiv) != [0, 1, 2] or L[2, 1] != -1.0 or U[2, 2] != 8.0:
        failed.append("tie_later_step")

    # exact rational elimination on small integer matrices without later ties
    tested = 0
    seed = 0
    while tested < 10 and seed < 200:
        A = gen.rng(1000 + seed).integers(-9, 10, size=(5, 5)).astype(np.float64)
        seed += 1
        Lq, Uq, pq, tie = exact_gepp(A)
        if tie or any(Uq[i][i] == 0 for i in range(5)):
            continue
        tested += 1
        L, U, ipiv, fail = lu_piv(A)
        scale = float(np.abs(A).max())
        ok = list(ipiv) == pq and fail == -1
        ok = ok and all(_close(L[i, c], Lq[i][c], 1.0, 1e-13) and
                        _close(U[i, c], Uq[i][c], scale, 1e-13)
                        for i in range(5) for c in range(5))
        if not ok:
            failed.append("exact_small")
            break

    # LAPACK's dgetrf (scipy.linalg.lu_factor): same exchanges, same factors
    import scipy.linalg as sl
    A = gen.rng(17).standard_normal((120, 120))
    L, U, ipiv, fail = lu_piv(A)
    lu, piv = sl.lu_factor(A)
    if (fail != -1 or not np.array_equal(ipiv, piv)
            or np.abs(np.tril(lu, -1) - np.tril(L, -1)).max() > 1e-12
            or np.abs(np.triu(lu) - U).max() > 1e-12 * np.abs(U).max()):
        failed.append("lapack")

    # invariants: |l_ij| <= 1 and P A = L U to rounding, also with zeros on
    # the diagonal (pivoting is required there)
    for A in (gen.rng(5).standard_normal((160, 160)),
              np.roll(np.eye(40) + 0.1 * gen.rng(6).standard_normal((40, 40)) * (1 - np.eye(40)),
                      1, axis=0)):
        n = A.shape[0]
        L, U, ipiv, fail = lu_piv(A)
        p = oracle.perm_from_ipiv(ipiv)
        resid = np.linalg.norm(A[p] - L @ U) / np.linalg.norm(A)
        if (fail != -1 or np.abs(np.tril(L, -1)).max() > 1.0 or resid > 8 * n * U64
                or not np.array_equal(np.triu(L, 1), np.zeros((n, n)))
                or not np.array_equal(np.diag(L), np.ones(n))):
            failed.append("invariants")
            break

    # the first zero pivot of a singular matrix (LAPACK's INFO - 1)
    A = gen.rng(8).standard_normal((6, 6))
    A[:, 2] = 0.0
    _, _, _, fail = lu_piv(A)
    _, _, _, fail0 = lu_piv(np.zeros((4, 4)))
    if fail != 2 or fail0 != 0:
        failed.append("singular")
    return failed
