"""GPU tests of the LU factorization with partial pivoting (P A = L U) against
the pivoted oracle: the same row exchanges (bitwise ipiv), L and U within
rounding of the oracle's, |l_ij| <= 1, P A = L U to rounding, exact cases
(permutation matrices, ties), singular matrices, ragged block and panel
edges, and solves A X = B through it."""
import numpy as np
import pytest

import oracle
from paper_1612_01855_amd import inputs as gen

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a ROCm device"
    return _t


@pytest.fixture(scope="module")
def T():
    from paper_1612_01855_amd import trsm
    return trsm


def gpu_lu(torch, T, A, nb=0):
    Ad = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    f = T.LUPiv(A.shape[0], nb, device=Ad.device)
    f.factor(Ad)
    st, idx = f.check()
    F = Ad.cpu().numpy()
    L = np.tril(F, -1) + np.eye(A.shape[0])
    U = np.triu(F)
    return L, U, f.ipiv.cpu().numpy(), st, idx, f


@pytest.mark.parametrize("n,nb", [(1, 0), (7, 0), (32, 0), (33, 32), (100, 64), (300, 0),
                                  (777, 128), (1000, 256), (2048, 512)])
def test_matches_pivoted_oracle(torch, T, n, nb):
    A = gen.rng(40 + n).standard_normal((n, n))
    L, U, ipiv, st, idx, f = gpu_lu(torch, T, A, nb)
    Lo, Uo, po, fail = oracle.lu_piv(A)
    print(f"n={n} nb={f.nb}: ipiv equal {np.array_equal(ipiv, po)}, "
          f"max |dL| {np.abs(L - Lo).max():.1e}, max |dU| {np.abs(U - Uo).max():.1e}", flush=True)
    assert st == T.OK and idx == -1 and fail == -1
    assert np.array_equal(ipiv, po)
    assert np.abs(L - Lo).max() <= 1e-11
    assert np.abs(U - Uo).max() <= 1e-11 * np.abs(Uo).max()
    assert np.abs(np.tril(L, -1)).max(initial=0.0) <= 1.0
    p = oracle.perm_from_ipiv(ipiv)
    assert np.linalg.norm(A[p] - L @ U) / np.linalg.norm(A) <= 8 * n * U64


def test_exact_cases_give_the_oracle_bits(torch, T):
    # scaled permutation matrices and ties resolve exactly as in the oracle
    g = gen.rng(5)
    for n in (5, 40, 300):
        A = np.zeros((n, n))
        A[g.permutation(n), np.arange(n)] = 2.0 ** g.integers(-3, 4, size=n)
        L, U, ipiv, st, _, _ = gpu_lu(torch, T, A)
        Lo, Uo, po, _ = oracle.lu_piv(A)
        assert st == T.OK
        assert np.array_equal(ipiv, po) and np.array_equal(L, Lo) and np.array_equal(U, Uo)
    for A in (np.array([[1.0, 5.0], [-1.0, 2.0]]),
              np.array([[4.0, 0.0, 0.0], [0.0, 1.0, 3.0], [0.0, -1.0, 5.0]]),
              np.kron(np.eye(20), np.array([[1.0, 2.0], [-1.0, 3.0]]))):
        L, U, ipiv, st, _, _ = gpu_lu(torch, T, A)
        Lo, Uo, po, _ = oracle.lu_piv(A)
        assert np.array_equal(ipiv, po) and np.array_equal(L, Lo) and np.array_equal(U, Uo)


def test_needs_pivoting(torch, T):
    # zero diagonal: LU without exchanges fails at the first step
    n = 500
    A = np.roll(np.eye(n), 1, axis=0) + 0.01 * gen.rng(7).standard_normal((n, n)) * \
        (1 - np.roll(np.eye(n), 1, axis=0))
    A[np.arange(n), np.arange(n)] = 0.0
    L, U, ipiv, st, _, _ = gpu_lu(torch, T, A)
    Lo, Uo, po, fail = oracle.lu_piv(A)
    assert st == T.OK and fail == -1
    assert np.array_equal(ipiv, po)
    p = oracle.perm_from_ipiv(ipiv)
    assert np.linalg.norm(A[p] - L @ U) / np.linalg.norm(A) <= 8 * n * U64


def test_singular_reports_first_zero_pivot(torch, T):
    n = 200
    A = gen.rng(9).standard_normal((n, n))
    A[:, 70] = 0.0
    A[:, 150] = 0.0
    _, _, ipiv, st, idx, _ = gpu_lu(torch, T, A)
    _, _, po, fail = oracle.lu_piv(A)
    assert st == T.ESINGULAR and idx == 70 == fail


def test_solve_through_pivoted_lu(torch, T):
    n, k = 1500, 40
    A = gen.rng(11).standard_normal((n, n))
    B = gen.rng(12).standard_normal((n, k))
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    X = T.lu_piv_solve(Ad, Bd).cpu().numpy()
    Lo, Uo, po, _ = oracle.lu_piv(A)
    Y = oracle.trsm(Lo, B[oracle.perm_from_ipiv(po)])
    Xo = oracle.trsm_t(np.ascontiguousarray(Uo.T), Y)
    berr = np.linalg.norm(A @ X - B) / (np.linalg.norm(A) * np.linalg.norm(X))
    err = oracle.rel_fro_err(X, Xo)
    print(f"solve n={n} k={k}: backward error {berr:.1e}, rel diff vs oracle {err:.1e}", flush=True)
    assert berr <= 8 * n * U64
    assert err <= 1e-9


def test_row_swaps_apply_ipiv(torch, T):
    n, k = 64, 9
    B = gen.rng(13).standard_normal((n, k))
    ipiv = np.array([min(n - 1, j + (j * 7) % 5) for j in range(n)], dtype=np.int64)
    Bd = torch.from_numpy(B.copy()).cuda()
    ip = torch.from_numpy(ipiv).cuda()
    T.trsm_row_swaps(0, n, ip.data_ptr(), Bd.data_ptr(), k, k,
                     torch.cuda.current_stream().cuda_stream)
    assert np.array_equal(Bd.cpu().numpy(), B[oracle.perm_from_ipiv(ipiv)])


def test_full_size_n16384_properties(torch, T):
    """n = 16384 (the solve's full size), where the oracle's O(n^3)
    elimination is out of reach: properties that hold at any size, |l_ij| <=
    1 and P A = L U to rounding (the product formed on the GPU), and a solve
    whose backward error is at binary64's level."""
    n, k = 16384, 16
    g = torch.Generator(device="cuda").manual_seed(17)
    A = torch.randn((n, n), generator=g, device="cuda", dtype=torch.float64)
    F = A.clone()
    f = T.LUPiv(n, 0, device=A.device)
    f.factor(F)
    torch.cuda.synchronize()
    st, idx = f.check()
    assert st == T.OK and idx == -1
    ipiv = f.ipiv.cpu().numpy()
    assert np.all(ipiv >= np.arange(n)) and np.all(ipiv < n)
    L = torch.tril(F, -1)
    L.diagonal().fill_(1.0)
    U = torch.triu(F)
    assert float(L.abs().max()) <= 1.0
    p = torch.from_numpy(oracle.perm_from_ipiv(ipiv)).cuda()
    rel = float(torch.linalg.norm(A[p] - L @ U) / torch.linalg.norm(A))
    del L, U
    B = torch.randn((n, k), generator=g, device="cuda", dtype=torch.float64)
    X = T.lu_piv_solve(A, B)
    berr = float(torch.linalg.norm(A @ X - B) / (torch.linalg.norm(A) * torch.linalg.norm(X)))
    print(f"n={n} nb={f.nb}: ||PA - LU|| / ||A|| = {rel:.2e}, solve backward error {berr:.1e}",
          flush=True)
    assert rel <= 8 * n * U64
    assert berr <= 8 * n * U64
