"""The oracle's Frobenius norms, relative forward error and normwise backward
error against closed forms, exact rationals and numpy (see norm_pins.py).
CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_1612_01855_amd import inputs as gen
from norm_pins import exact_sumsq, failed_norm_pins, sqrt_rounded


def test_every_norm_pin_holds():
    assert failed_norm_pins(oracle) == []


@pytest.mark.parametrize("n", [1, 2, 9, 16, 333])
def test_identity_and_ones_closed_forms(n):
    eye = gen.identity(n)
    eye[np.triu_indices(n, 1)] = np.nan
    assert oracle.fro_lower(eye) == math.sqrt(n)
    ones = gen.ones_lower(n)
    ones[np.triu_indices(n, 1)] = np.nan
    assert oracle.fro_lower(ones) == math.sqrt(n * (n + 1) // 2)


def test_lower_norm_ignores_upper_triangle_and_counts_diagonal():
    L = gen.rng(3).normal(size=(7, 7))
    tri = np.tril(L)
    ref = sqrt_rounded(exact_sumsq(tri[np.tril_indices(7)]))
    L2 = L.copy()
    L2[np.triu_indices(7, 1)] = 1e300
    assert oracle.fro_lower(L2) == oracle.fro_lower(tri)
    assert abs(oracle.fro_lower(tri) - ref) <= math.ulp(ref)
    # dropping the diagonal would change the norm by at least this much
    no_diag = sqrt_rounded(exact_sumsq(L[np.tril_indices(7, -1)]))
    assert oracle.fro_lower(tri) - no_diag > 1e3 * math.ulp(ref)


def test_empty_and_zero():
    assert oracle.fro(np.zeros((5, 3))) == 0.0
    assert oracle.fro_lower(np.zeros((4, 4))) == 0.0
    X = np.zeros((3, 2))
    assert oracle.rel_fro_err(X, X) == 0.0
