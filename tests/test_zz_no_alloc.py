"""trsm_solve_noalloc, the allocation-free solve (workspace in a static
device array): its X must match trsm_solve's on the same plan and inverted
blocks, to the binary64 / binary32 parity bar, on two calls in a row (the
second smaller), and both must match the oracle.  The size and mode checks
run before any device work, so they are CPU tests."""
import numpy as np
import pytest

import oracle
from paper_1612_01855_amd import inputs as gen


@pytest.fixture(scope="module")
def T():
    from paper_1612_01855_amd import trsm
    return trsm


def test_noalloc_rejects_oversized_and_unsupported_plans(T):
    cap = T.trsm_solve_noalloc_max_bytes()
    assert cap == 2 << 20
    # n * k binary64 values beyond the static array: refused before any device work
    big = T.trsm_plan(4096, 4096, T.F64, 0, 0)
    try:
        assert T.trsm_solve_noalloc(big, 1, 4096, 256, 1, 4096, 2, 4096, 0) == T.ENOMEM
    finally:
        T.trsm_plan_destroy(big)
    # mixed precision and lookahead plans keep their own workspaces
    for prec, flags in ((T.MIXED_F16, 0), (T.F64, T.FLAG_LOOKAHEAD)):
        p = T.trsm_plan(256, 64, prec, 0, flags)
        try:
            assert T.trsm_solve_noalloc(p, 1, 256, 256, 1, 64, 2, 64, 0) == T.EINVAL
        finally:
            T.trsm_plan_destroy(p)
    assert T.trsm_solve_noalloc(0, 1, 1, 256, 1, 1, 2, 1, 0) == T.EINVAL


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_matches_trsm_solve_twice(T, prec):
    import torch
    assert torch.cuda.is_available()
    dt = torch.float64 if prec == "f64" else torch.float32
    tol = 1e-12 if prec == "f64" else 1e-5
    # the second call is smaller: the array keeps the first call's contents
    for n, k, n0, seed in ((600, 400, 128, 71), (300, 37, 64, 72)):
        L, B = gen.easy_system(n, k, seed, upper=np.nan)
        if prec == "f32":
            L, B = L.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
        Ld = torch.from_numpy(L).to("cuda", dt)
        Bd = torch.from_numpy(B).to("cuda", dt)
        s = T.Solver.create(n, k, prec, n0)
        try:
            s.invert(Ld)
            X_ref = s.solve(Ld, Bd)
            X_na = torch.full_like(Bd, float("nan"))
            stream = torch.cuda.current_stream().cuda_stream
            st = T.trsm_solve_noalloc(s.plan, Ld.data_ptr(), n, s.linv_ptr, Bd.data_ptr(), k,
                                      X_na.data_ptr(), k, stream)
            torch.cuda.synchronize()
            assert st == T.OK, T.status_string(st)
        finally:
            s.close()
        Xr = X_ref.double().cpu().numpy()
        Xn = X_na.double().cpu().numpy()
        Xo = oracle.trsm(L, B)
        d = oracle.rel_fro_err(Xn, Xr)
        e = oracle.rel_fro_err(Xn, Xo)
        print(f"{prec} n={n} k={k}: no-alloc vs trsm_solve {d:.2e}, vs oracle {e:.2e}", flush=True)
        assert np.isfinite(Xn).all()
        assert d <= tol
        assert e <= tol
