"""Exact rational arithmetic for brute-force pins -- TEST INFRASTRUCTURE ONLY.

Everything here works on Python ``fractions.Fraction`` values, so results are
exact.  It is deliberately a different algorithm from the forward substitution
in ``oracle.c``: the inverse is found by Gauss-Jordan elimination on the
augmented matrix [L | I] over the rationals, treating L as a general square
matrix (the triangular structure is not used).  A transposed operand, a wrong
index or a dropped term in the substitution therefore cannot be reproduced
here by the same mistake.

Every binary64 number is a dyadic rational, so ``Fraction(float)`` is exact.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence

Matrix = List[List[Fraction]]


def to_q(a) -> Matrix:
    """Convert a 2-D array-like of floats/ints to an exact rational matrix."""
    return [[Fraction(float(v)) if not isinstance(v, (int, Fraction)) else Fraction(v)
             for v in row] for row in a]


def lower_part(a: Matrix) -> Matrix:
    """Keep the lower triangle (diagonal included), zero above it: the only
    entries of L the problem statement uses."""
    n = len(a)
    return [[a[i][j] if j <= i else Fraction(0) for j in range(n)] for i in range(n)]


def inverse(a: Matrix) -> Matrix:
    """Inverse of a general nonsingular square matrix by Gauss-Jordan
    elimination with row pivoting on the first nonzero entry, over Q."""
    n = len(a)
    aug = [list(a[i]) + [Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for col in range(n):
        piv = next((r for r in range(col, n) if aug[r][col] != 0), None)
        if piv is None:
            raise ZeroDivisionError("singular matrix")
        aug[col], aug[piv] = aug[piv], aug[col]
        p = aug[col][col]
        aug[col] = [v / p for v in aug[col]]
        for r in range(n):
            if r != col and aug[r][col] != 0:
                f = aug[r][col]
                aug[r] = [vr - f * vc for vr, vc in zip(aug[r], aug[col])]
    return [row[n:] for row in aug]


def matmul(a: Matrix, b: Matrix) -> Matrix:
    n, m, k = len(a), len(b), len(b[0]) if b else 0
    return [[sum((a[i][p] * b[p][j] for p in range(m)), Fraction(0)) for j in range(k)]
            for i in range(n)]


def absm(a: Matrix) -> Matrix:
    return [[abs(v) for v in row] for row in a]


def solve(L, B) -> Matrix:
    """Exact X = L^{-1} B over Q, with L's upper triangle ignored."""
    Lq = lower_part(to_q(L))
    return matmul(inverse(Lq), to_q(B))


def substitution_bound(L, Xhat, n_ops: int) -> Matrix:
    """Componentwise first-order forward-error bound of forward substitution
    (the standard backward-error result for triangular solves: the computed
    solution solves (L + dL) x = b with |dL| <= gamma_n |L|, gamma_n =
    n u / (1 - n u), u = 2^-53), turned into a forward bound
    |x - xhat| <= gamma_n |L^{-1}| |L| |xhat| evaluated exactly."""
    u = Fraction(1, 2 ** 53)
    g = n_ops * u / (1 - n_ops * u)
    Lq = lower_part(to_q(L))
    Linv = inverse(Lq)
    M = matmul(matmul(absm(Linv), absm(Lq)), absm(to_q(Xhat)))
    return [[g * v for v in row] for row in M]


def is_integer_matrix(a: Matrix) -> bool:
    return all(v.denominator == 1 for row in a for v in row)


def to_float(a: Matrix):
    return [[float(v) for v in row] for row in a]


def max_abs(a: Sequence[Sequence[Fraction]]) -> Fraction:
    return max((abs(v) for row in a for v in row), default=Fraction(0))
