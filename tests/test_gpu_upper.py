"""GPU parity of the upper-triangular solve U X = B (TRSM_FLAG_UPPER: the
backward sweep of Alg. It-Inv-TRSM over U read in place, with U's inverted
diagonal blocks) through the C ABI against the CPU oracle's backward
substitution, on the same seeded inputs.  The oracle solves L^T X = B for a
lower L, so it is given L = U^T; the GPU is given U with NaN below its
diagonal, which it must never read.  Tolerances: 1e-12 relative Frobenius
error in binary64, 1e-5 in binary32 (oracle on the binary32-rounded inputs).
Last, the whole LU solve A X = B on the GPU: the LU factorization without row
exchanges, L Y = B with its inverted blocks, then U X = Y on the factored A
in place."""
import numpy as np
import pytest

import oracle
from paper_1612_01855_amd import inputs as gen

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a ROCm device"
    return _t


@pytest.fixture(scope="module")
def T():
    from paper_1612_01855_amd import trsm
    return trsm


def log(msg):
    print(msg, flush=True)


def upper_system(n, k, seed):
    """(U with NaN below the diagonal, L = U^T clean for the oracle, B)."""
    L, B = gen.easy_system(n, k, seed)
    U = np.ascontiguousarray(L.T)
    U[np.tril_indices(n, -1)] = np.nan
    return U, L, B


def gpu_upper(torch, T, U, B, precision="f64", n0=0, inplace=False):
    n, k = B.shape
    dt = torch.float32 if precision == "f32" else torch.float64
    Ud = torch.from_numpy(U).to("cuda", dt)
    Bd = torch.from_numpy(B).to("cuda", dt)
    s = T.Solver.create(n, k, precision, n0, T.FLAG_UPPER)
    log(f"upper n={n} k={k} {precision} n0={s.info.n0} inplace={inplace}")
    try:
        s.invert(Ud)
        X = s.solve(Ud, Bd, Bd if inplace else None)
        torch.cuda.synchronize()
        assert s.last_error() == (T.OK, -1)
        return X.to(torch.float64).cpu().numpy()
    finally:
        s.close()


@pytest.mark.parametrize("n,k,n0", [(1, 1, 0), (7, 3, 0), (100, 3, 32), (1000, 70, 128),
                                    (1537, 40, 256), (2048, 64, 0), (600, 1, 64)])
def test_upper_matches_oracle(torch, T, n, k, n0):
    U, L, B = upper_system(n, k, n + k)
    X = gpu_upper(torch, T, U, B, "f64", n0)
    err = oracle.rel_fro_err(X, oracle.trsm_t(L, B))
    log(f"  rel err {err:.2e}")
    assert err <= TOL64


def test_upper_in_place(torch, T):
    U, L, B = upper_system(700, 20, 3)
    X = gpu_upper(torch, T, U, B, "f64", 128, inplace=True)
    assert oracle.rel_fro_err(X, oracle.trsm_t(L, B)) <= TOL64


def test_upper_f32_against_oracle_on_rounded_inputs(torch, T):
    U, L, B = upper_system(513, 40, 5)
    L32 = L.astype(np.float32).astype(np.float64)
    B32 = B.astype(np.float32).astype(np.float64)
    X = gpu_upper(torch, T, U.astype(np.float32), B.astype(np.float32), "f32", 64)
    err = oracle.rel_fro_err(X, oracle.trsm_t(L32, B32))
    log(f"  f32 rel err {err:.2e}")
    assert err <= TOL32


def test_upper_closed_form_is_exact(torch, T):
    # U = I - (superdiagonal of ones): U^{-1} is the all-ones upper triangle,
    # so X_i = sum_{j >= i} B_j (suffix sums); with small integers every
    # product and sum is exact and X must come back bit for bit
    n, k = 1000, 5
    U = np.eye(n) - np.eye(n, k=1)
    U[np.tril_indices(n, -1)] = np.nan
    B = gen.rng(17).integers(-3, 4, size=(n, k)).astype(np.float64)
    expect = np.cumsum(B[::-1], axis=0)[::-1]
    for n0 in (32, 128, 512):
        X = gpu_upper(torch, T, U, B, "f64", n0)
        assert np.array_equal(X, expect), n0


def test_upper_singular_reports_the_row(torch, T):
    U, _, _ = upper_system(300, 3, 9)
    U[137, 137] = 0.0
    U[150, 150] = np.nan
    s = T.Solver.create(300, 3, "f64", 64, T.FLAG_UPPER)
    try:
        s.invert(torch.from_numpy(U).cuda())
        torch.cuda.synchronize()
        assert s.last_error() == (T.ESINGULAR, 137)
    finally:
        s.close()


@pytest.mark.parametrize("n,k,nb", [(1100, 40, 256), (2048, 17, 512)])
def test_lu_solve_on_the_gpu(torch, T, n, k, nb):
    A = gen.diag_dominant(n, n + 3)
    B = gen.rhs(n, k, n + 3)
    Ad = torch.from_numpy(A.copy()).cuda()
    f = T.LU(n, nb, device="cuda")
    f.factor(Ad)
    fwd = T.Solver.create(n, k, "f64", n0=nb)
    up = T.Solver.create(n, k, "f64", 0, T.FLAG_UPPER)
    try:
        # L Y = B with the factorization's own inverted blocks (unit diagonal stored)
        Bd = torch.from_numpy(B).cuda()
        Yd = torch.empty_like(Bd)
        T.trsm_solve(fwd.plan, Ad.data_ptr(), n, f.linv_ptr, Bd.data_ptr(), k, Yd.data_ptr(), k,
                     fwd.workspace_ptr, torch.cuda.current_stream().cuda_stream, None)
        # U X = Y on the factored A: U is its upper triangle, L below is not read
        up.invert(Ad)
        Xd = up.solve(Ad, Yd)
        torch.cuda.synchronize()
        assert f.check() == (T.OK, -1)
        assert up.last_error() == (T.OK, -1)
    finally:
        fwd.close()
        up.close()
    X = Xd.cpu().numpy()
    F = Ad.cpu().numpy()
    Lf = np.tril(F, -1) + np.eye(n)
    Uf = np.triu(F)
    ref = oracle.trsm_t(np.ascontiguousarray(Uf.T), oracle.trsm(Lf, B))
    err_chain = oracle.rel_fro_err(X, ref)
    err_a = oracle.rel_fro_err(X, np.linalg.solve(A, B))
    log(f"  lu solve n={n}: vs oracle chain {err_chain:.2e}, vs A^-1 B {err_a:.2e}")
    assert err_chain <= TOL64 and err_a <= TOL64


def test_lu_solve_helper(torch, T):
    n, k = 900, 12
    A = gen.diag_dominant(n, 77)
    B = gen.rhs(n, k, 77)
    X = T.lu_solve(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), nb=128)
    err = oracle.rel_fro_err(X.cpu().numpy(), np.linalg.solve(A, B))
    log(f"  lu_solve helper: rel err {err:.2e}")
    assert err <= TOL64
    A[300, 300] = np.nan
    with pytest.raises(T.TrsmError):
        T.lu_solve(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), nb=128)


@pytest.mark.parametrize("n,nb", [(100, 256), (65, 0), (1000, 1024)])
def test_lu_solve_block_size_beyond_the_matrix(torch, T, n, nb):
    # a requested block larger than the next power of two >= n is cut to it,
    # the cap a plan puts on n0, so the inverted blocks keep the plan's layout
    A = gen.diag_dominant(n, 31)
    B = gen.rhs(n, 3, 31)
    X = T.lu_solve(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), nb=nb)
    err = oracle.rel_fro_err(X.cpu().numpy(), np.linalg.solve(A, B))
    log(f"  lu_solve n={n} nb={nb}: rel err {err:.2e}")
    assert err <= 1e-12


@pytest.mark.parametrize("n", [1, 20])
def test_lu_solve_refuses_blocks_a_plan_cannot_read(torch, T, n):
    # below n = 33 a plan's n0 is under the factorization's 64-row leaf: the
    # helper refuses instead of reading the blocks with the wrong row stride
    A = gen.diag_dominant(n, 32)
    B = gen.rhs(n, 2, 32)
    with pytest.raises(ValueError):
        T.lu_solve(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda())
