"""Pins for the CPU oracle, checked against facts that do not come from the
oracle itself: closed-form inverses, exact rational arithmetic (Gauss-Jordan
on Q, a different algorithm), the standard error bound of forward
substitution, the residual postcondition B = L X of Alg. It-Inv-TRSM, and the
independence of right-hand-side columns (Sec. II-C.4).  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import exact
from paper_1612_01855_amd import inputs as gen

NAN = float("nan")


# ---- closed forms ----------------------------------------------------------

@pytest.mark.parametrize("n,k", [(1, 1), (7, 3), (64, 5), (200, 17)])
def test_identity_gives_b_bitwise(n, k):
    L = gen.identity(n)
    L[np.triu_indices(n, 1)] = NAN
    B = gen.rhs(n, k, seed=1)
    X = oracle.trsm(L, B)
    assert np.array_equal(X, B)


@pytest.mark.parametrize("n,k", [(1, 4), (33, 9), (150, 2)])
def test_diagonal_gives_one_rounded_division(n, k):
    L = gen.diagonal(n, seed=2)
    d = np.diag(L).copy()
    L[np.triu_indices(n, 1)] = NAN
    B = gen.rhs(n, k, seed=3)
    X = oracle.trsm(L, B)
    assert np.array_equal(X, B / d[:, None])


@pytest.mark.parametrize("n,k", [(2, 1), (9, 4), (300, 11)])
def test_bidiagonal_gives_prefix_sums(n, k):
    # L^{-1} is the all-ones lower triangle: x_i = b_i + x_{i-1}, i.e. the
    # running column sum, which numpy's cumsum forms in the same order.
    L = gen.bidiagonal_minus_one(n)
    L[np.triu_indices(n, 1)] = NAN
    B = gen.rhs(n, k, seed=4)
    X = oracle.trsm(L, B)
    assert np.array_equal(X, np.cumsum(B, axis=0))


@pytest.mark.parametrize("n,k", [(1, 1), (8, 3), (257, 6)])
def test_ones_lower_gives_differences(n, k):
    # L^{-1} is unit lower bidiagonal with -1 below the diagonal.
    L = gen.ones_lower(n)
    L[np.triu_indices(n, 1)] = NAN
    B = gen.int_rhs(n, k, seed=5)
    X = oracle.trsm(L, B)
    expect = B.copy()
    expect[1:] -= B[:-1]
    assert np.array_equal(X, expect)


# ---- exact rational brute force ---------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_within_substitution_bound(n, seed):
    L, B = gen.easy_system(n, 3, seed)
    L[np.triu_indices(n, 1)] = NAN
    X = oracle.trsm(L, B)
    Xq = exact.solve(np.nan_to_num(L, nan=0.0), B)
    bound = exact.substitution_bound(np.nan_to_num(L, nan=0.0), X, n_ops=n + 1)
    for i in range(n):
        for c in range(3):
            err = abs(exact.Fraction(float(X[i, c])) - Xq[i][c])
            assert err <= bound[i][c], (i, c, float(err), float(bound[i][c]))


@pytest.mark.parametrize("n", [4, 8])
def test_brute_force_general_scale(n):
    # entries of mixed magnitude and sign, not diagonally dominant
    g = gen.rng(11)
    L = np.tril(g.standard_normal((n, n)))
    L[np.arange(n), np.arange(n)] = g.uniform(0.5, 2.0, n) * g.choice([-1.0, 1.0], n)
    B = g.standard_normal((n, 2)) * 1e3
    X = oracle.trsm(L, B)
    Xq = exact.solve(L, B)
    bound = exact.substitution_bound(L, X, n_ops=n + 1)
    for i in range(n):
        for c in range(2):
            assert abs(exact.Fraction(float(X[i, c])) - Xq[i][c]) <= bound[i][c]


@pytest.mark.parametrize("n,seed", [(8, 0), (16, 1), (24, 2), (40, 3)])
def test_integer_unit_lower_inverse_is_exact(n, seed):
    L = gen.int_unit_lower(n, seed)
    Linv_q = exact.inverse(exact.to_q(L))
    assert exact.is_integer_matrix(Linv_q)
    if exact.max_abs(Linv_q) >= 2 ** 53:
        pytest.skip("inverse entries exceed 2^53")
    Linv = oracle.inv_lower(L)
    assert np.array_equal(Linv, np.array(exact.to_float(Linv_q)))


def test_integer_solution_recovered_exactly():
    n, k = 48, 5
    L = gen.int_unit_lower(n, 9, density=0.3)
    Xtrue = gen.int_rhs(n, k, 9, -3, 3)
    B = L @ Xtrue                      # small integers: exact in binary64
    assert np.abs(B).max() < 2 ** 40
    assert np.array_equal(oracle.trsm(L, B), Xtrue)


def test_quad_oracle_matches_exact_rational():
    n = 8
    L, B = gen.easy_system(n, 2, 5)
    Xq = exact.solve(L, B)
    Xquad = oracle.trsm_q(L, B)
    for i in range(n):
        for c in range(2):
            ref = Xq[i][c]
            err = abs(exact.Fraction(float(Xquad[i, c])) - ref)
            assert err <= abs(ref) * exact.Fraction(1, 2 ** 52)


def test_residual_matches_exact_rational():
    n, k = 7, 3
    L, B = gen.easy_system(n, k, 6)
    X = oracle.trsm(L, B) + 1e-3     # a perturbed X gives a sizeable residual
    R = oracle.residual(L, X, B)
    Rq = [[exact.Fraction(float(B[i, c]))
           - sum((exact.Fraction(float(L[i, j])) * exact.Fraction(float(X[j, c]))
                  for j in range(i + 1)), exact.Fraction(0))
           for c in range(k)] for i in range(n)]
    u = exact.Fraction(1, 2 ** 53)
    for i in range(n):
        for c in range(k):
            scale = abs(exact.Fraction(float(B[i, c]))) + sum(
                abs(exact.Fraction(float(L[i, j])) * exact.Fraction(float(X[j, c])))
                for j in range(i + 1))
            assert abs(exact.Fraction(float(R[i, c])) - Rq[i][c]) <= 2 * (n + 2) * u * scale


# ---- postcondition and structure --------------------------------------------

@pytest.mark.parametrize("gen_name,n,k", [("easy", 256, 64), ("easy", 1000, 33),
                                          ("chol", 384, 48), ("chol", 129, 200)])
def test_residual_invariant(gen_name, n, k):
    if gen_name == "easy":
        L = gen.easy_lower(n, 0, upper=NAN)
    else:
        L = gen.chol_lower(n, 0, upper=NAN)
    B = gen.rhs(n, k, 0)
    X = oracle.trsm(L, B)
    assert oracle.backward_err(L, X, B) <= 1e-14


def test_column_split_is_bitwise_and_thread_invariant():
    n, k = 300, 150
    L, B = gen.easy_system(n, k, 7)
    X = oracle.trsm(L, B)
    X1 = oracle.trsm(L, B[:, :70])
    X2 = oracle.trsm(L, B[:, 70:])
    assert np.array_equal(X, np.hstack([X1, X2]))
    assert np.array_equal(X, oracle.trsm(L, B, nthreads=1))
    assert np.array_equal(X, oracle.trsm(L, B, nthreads=3))


def test_in_place_and_strided_views():
    n, k = 90, 12
    L, B = gen.easy_system(n, k, 8)
    Lbig = np.full((n, n + 5), NAN)
    Lbig[:, :n] = np.tril(L)
    Lbig[:, :n][np.triu_indices(n, 1)] = NAN
    X = oracle.trsm(L, B)
    assert np.array_equal(oracle.trsm(Lbig[:, :n], B), X)
    Bbig = np.zeros((n, k + 3))
    Bbig[:, :k] = B
    assert np.array_equal(oracle.trsm(L, Bbig[:, :k]), X)


def test_block_inverses_postcondition():
    n, n0 = 200, 64                  # ragged last block of 8
    L = gen.easy_lower(n, 3, upper=NAN)
    invs = oracle.diag_block_inverses(L, n0)
    assert [a.shape[0] for a in invs] == [64, 64, 64, 8]
    for b, Ainv in enumerate(invs):
        s = b * n0
        blk = np.tril(np.nan_to_num(L[s:s + Ainv.shape[0], s:s + Ainv.shape[0]]))
        assert np.abs(Ainv @ blk - np.eye(blk.shape[0])).max() < 1e-14
        assert np.all(np.triu(Ainv, 1) == 0)


def test_hard_matrix_is_ill_conditioned_and_oracle_accurate():
    n, k = 256, 4
    L = gen.hard_lower(n, 0)
    c = np.linalg.cond(L)
    assert 1e4 < c < 1e8
    B = gen.rhs(n, k, 0)
    X = oracle.trsm(L, B)
    Xq = oracle.trsm_q(L, B)
    assert oracle.rel_fro_err(X, Xq) <= c * n * 2.0 ** -52
    assert oracle.backward_err(L, X, B) <= 1e-15


def test_empty_sizes():
    assert oracle.trsm(np.eye(3), np.zeros((3, 0))).shape == (3, 0)
    assert oracle.trsm(np.zeros((0, 0)), np.zeros((0, 4))).shape == (0, 4)


# ---- golden fixtures (exact rational values written by tests/golden) --------

def test_golden_integer_inverse():
    from golden_io import load
    g = load("int_unit_lower_n10.txt")
    assert np.array_equal(oracle.inv_lower(g["L"]), g["Linv"])


@pytest.mark.parametrize("name", ["easy_n6_k3.txt", "hard_n8_k2.txt"])
def test_golden_exact_solution(name):
    from golden_io import load
    g = load(name)
    L, B, Xexact = g["L"], g["B"], g["X"]
    X = oracle.trsm(L, B)
    n = L.shape[0]
    bound = exact.substitution_bound(L, X, n_ops=n + 1)
    for i in range(n):
        for c in range(B.shape[1]):
            # |X - Xexact_rounded| <= bound + half an ulp of the rounding
            err = abs(exact.Fraction(float(X[i, c])) - exact.Fraction(float(Xexact[i, c])))
            assert err <= bound[i][c] + exact.Fraction(abs(float(Xexact[i, c]))) * exact.Fraction(1, 2 ** 53)
    # the quad-precision oracle rounds to the same binary64 values
    assert np.abs(oracle.trsm_q(L, B) - Xexact).max() <= 2.0 ** -52 * np.abs(Xexact).max()
