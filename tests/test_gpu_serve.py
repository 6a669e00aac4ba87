"""GPU tests of the continuous-batching server: every request matches the
oracle on its own (L, B) (gate 1e-12), each request's refinement stops by its
own test and reports its trsm_info, a request's result and info are bitwise
the same alone and in a mix, admission respects the HBM budget, the
correction cap ends a request with TRSM_ENOTCONVERGED, and an impossible
request fails cleanly."""
import time

import numpy as np
import pytest

import oracle
from paper_1612_01855_amd import inputs as gen

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a ROCm device"
    return _t


@pytest.fixture(scope="module")
def T():
    from paper_1612_01855_amd import trsm
    return trsm


def wait_all(T, srv, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    pending = set(tickets)
    while pending:
        for t in list(pending):
            st, status, info = T.trsm_serve_poll(srv, t)
            if st in (T.REQ_DONE, T.REQ_ERROR):
                out[t] = (st, status, info)
                pending.discard(t)
        assert time.time() - t0 < timeout, "server did not finish in time"
        time.sleep(0.0005)
    return out


def info_tuple(info):
    return (info.iterations, info.converged, info.backward_error, info.correction,
            info.unrefined_error)


def check_info(info, n, precision):
    """The stopping test the server applies, restated: converged requests
    have a backward error within sqrt(n) u or a correction that stopped
    mattering."""
    assert info.converged == 1
    if precision == "f32":
        assert info.iterations >= 1 and info.unrefined_error > 0
    stalled = info.correction >= 0 and info.correction <= 1e-15
    assert info.backward_error <= np.sqrt(n) * U or stalled or info.iterations >= 2


def submit(T, srv, lid, q):
    return T.trsm_serve_submit(srv, lid, q["Bd"].data_ptr(), q["k"], q["k"],
                               q["Xd"].data_ptr(), q["k"])


@pytest.mark.parametrize("n0,precision", [(0, "f32"), (128, "f32"), (64, "f32"), (0, "f64"),
                                          (64, "f64")])
def test_server_requests_match_oracle_and_mix_independence(torch, T, n0, precision):
    # n0 = 0: the default (factors up to 4096 rows inverted whole); 64:
    # persistent sweeps
    srv = T.trsm_server_create(2 << 30, 32, n0)
    try:
        ns = [64, 200, 777, 1300]
        Ls, lids = [], []
        for i, n in enumerate(ns):
            L = gen.easy_lower(n, 100 + i, upper=np.nan)
            Ld = torch.from_numpy(L).cuda()
            lids.append(T.trsm_server_register_L(srv, Ld.data_ptr(), n, n, precision))
            Ls.append(L)
            del Ld
        torch.cuda.synchronize()
        g = gen.rng(5)
        reqs = []
        for r in range(16):
            f = int(g.integers(0, len(ns)))
            k = int(gen.log_uniform_int(g, 1, 300))
            B = gen.rhs(ns[f], k, 300 + r)
            Bd = torch.from_numpy(B).cuda()
            Xd = torch.full_like(Bd, float("nan"))
            reqs.append(dict(f=f, k=k, B=B, Bd=Bd, Xd=Xd))
        torch.cuda.synchronize()
        tickets = [submit(T, srv, lids[q["f"]], q) for q in reqs]
        res = wait_all(T, srv, tickets)
        mix = []
        for q, t in zip(reqs, tickets):
            st, status, info = res[t]
            assert st == T.REQ_DONE and status == T.OK
            X = q["Xd"].cpu().numpy()
            n = ns[q["f"]]
            err = oracle.rel_fro_err(X, oracle.trsm(Ls[q["f"]], q["B"]))
            berr = oracle.backward_err(Ls[q["f"]], X, q["B"])
            print(f"request n={n} k={q['k']}: rel err {err:.2e}, berr {berr:.1e} "
                  f"(server {info.backward_error:.1e}), {info.iterations} corrections",
                  flush=True)
            assert err <= 1e-12
            check_info(info, n, precision)
            assert berr <= 4 * np.sqrt(n) * U
            mix.append((X.copy(), info_tuple(info)))
        # the same requests one at a time give the same bits and the same info
        for q, (X, inf) in zip(reqs[:6], mix[:6]):
            q["Xd"].fill_(float("nan"))
            torch.cuda.synchronize()
            t = submit(T, srv, lids[q["f"]], q)
            st, status, info = wait_all(T, srv, [t])[t]
            assert st == T.REQ_DONE and status == T.OK
            assert np.array_equal(q["Xd"].cpu().numpy(), X)
            assert info_tuple(info) == inf
        stats = T.trsm_server_stats(srv)
        assert stats.completed == 22 and stats.failed == 0 and stats.unconverged == 0
        assert stats.passes >= 22
        assert stats.p99_us >= stats.p50_us > 0
    finally:
        T.trsm_server_destroy(srv)


@pytest.mark.parametrize("n0", [128, 64])
def test_admission_respects_budget(torch, T, n0):
    n, k = 1024, 64
    # one factor (~12.6 MB and its registration's temporaries) plus room for
    # about two and a half requests
    probe = T.trsm_server_create(1 << 30, 4, n0)
    try:
        L = gen.easy_lower(n, 7, upper=np.nan)
        Ld = torch.from_numpy(L).cuda()
        T.trsm_server_register_L(probe, Ld.data_ptr(), n, n)
        per_req = T.trsm_serve_request_bytes(probe, 0, k)
        resident = T.trsm_server_stats(probe).resident_bytes
    finally:
        T.trsm_server_destroy(probe)
    assert 32 * n * k <= per_req <= 32 * n * k + max(64 * n * k, 4 << 20) + (1 << 20)
    budget = resident + (5 * per_req) // 2
    srv = T.trsm_server_create(budget, 64, n0)
    try:
        lid = T.trsm_server_register_L(srv, Ld.data_ptr(), n, n)
        reqs = []
        for r in range(12):
            B = gen.rhs(n, k, 50 + r)
            Bd = torch.from_numpy(B).cuda()
            reqs.append((B, Bd, torch.empty_like(Bd)))
        torch.cuda.synchronize()
        ts = [T.trsm_serve_submit(srv, lid, Bd.data_ptr(), k, k, Xd.data_ptr(), k)
              for _, Bd, Xd in reqs]
        res = wait_all(T, srv, ts)
        for (B, _, Xd), t in zip(reqs, ts):
            assert res[t][0] == T.REQ_DONE and res[t][1] == T.OK
            assert oracle.rel_fro_err(Xd.cpu().numpy(), oracle.trsm(L, B)) <= 1e-12
        stats = T.trsm_server_stats(srv)
        assert stats.resident_bytes == resident
        assert stats.max_in_flight * per_req <= budget - stats.resident_bytes
        assert stats.max_in_flight == 2
        print(f"budget {budget >> 20} MiB: at most {stats.max_in_flight} requests in flight",
              flush=True)
        # a request that can never fit fails instead of waiting forever
        kb = 4096
        Bd = torch.zeros((n, kb), dtype=torch.float64, device="cuda")
        Xd = torch.empty_like(Bd)
        t = T.trsm_serve_submit(srv, lid, Bd.data_ptr(), kb, kb, Xd.data_ptr(), kb)
        st, status, _ = wait_all(T, srv, [t])[t]
        assert st == T.REQ_ERROR and status == T.ENOMEM
    finally:
        T.trsm_server_destroy(srv)


@pytest.mark.parametrize("n0,precision", [(128, "f32"), (0, "f32"), (0, "f64")])
def test_cholesky_factors_mixed_with_triangular_ones(torch, T, n0, precision):
    # factors registered as Cholesky factors answer A X = B with A = L L^T;
    # triangular and Cholesky requests share batches
    srv = T.trsm_server_create(2 << 30, 32, n0)
    try:
        spec = [(150, True), (600, False), (1100, True), (333, True), (3000, True)]
        Ls, lids = [], []
        for i, (n, chol) in enumerate(spec):
            L = gen.chol_lower(n, 200 + i, upper=np.nan) if chol else \
                gen.easy_lower(n, 200 + i, upper=np.nan)
            Ld = torch.from_numpy(L).cuda()
            reg = T.trsm_server_register_chol if chol else T.trsm_server_register_L
            lids.append(reg(srv, Ld.data_ptr(), n, n, precision))
            Ls.append(L)
            del Ld
        torch.cuda.synchronize()
        g = gen.rng(9)
        reqs = []
        for r in range(14):
            f = int(g.integers(0, len(spec)))
            k = int(gen.log_uniform_int(g, 1, 200))
            B = gen.rhs(spec[f][0], k, 700 + r)
            Bd = torch.from_numpy(B).cuda()
            reqs.append(dict(f=f, k=k, B=B, Bd=Bd, Xd=torch.full_like(Bd, float("nan"))))
        torch.cuda.synchronize()
        tickets = [submit(T, srv, lids[q["f"]], q) for q in reqs]
        res = wait_all(T, srv, tickets)
        mix = []
        for q, t in zip(reqs, tickets):
            st, status, info = res[t]
            assert st == T.REQ_DONE and status == T.OK
            L = Ls[q["f"]]
            chol = spec[q["f"]][1]
            ref = oracle.trsm_t(L, oracle.trsm(L, q["B"])) if chol else oracle.trsm(L, q["B"])
            X = q["Xd"].cpu().numpy()
            err = oracle.rel_fro_err(X, ref)
            print(f"{'cholesky' if chol else 'triangular'} n={spec[q['f']][0]} "
                  f"k={q['k']}: rel err {err:.2e}, {info.iterations} corrections, "
                  f"berr {info.backward_error:.1e}", flush=True)
            assert err <= 1e-12
            assert info.converged == 1
            mix.append((X.copy(), info_tuple(info)))
        for q, (X, inf) in zip(reqs[:5], mix[:5]):
            q["Xd"].fill_(float("nan"))
            torch.cuda.synchronize()
            t = submit(T, srv, lids[q["f"]], q)
            st, status, info = wait_all(T, srv, [t])[t]
            assert st == T.REQ_DONE and status == T.OK
            assert np.array_equal(q["Xd"].cpu().numpy(), X)
            assert info_tuple(info) == inf
    finally:
        T.trsm_server_destroy(srv)


def test_concurrent_submitters_and_registration(torch, T):
    """Four host threads submit and poll at once while a fifth registers a new
    factor; every request's X is bitwise its lone result (computed first,
    one request at a time) and within 1e-12 of the oracle."""
    import threading
    srv = T.trsm_server_create(2 << 30, 16, 128)
    try:
        ns = [96, 333, 700]
        Ls, lids = [], []
        for i, n in enumerate(ns):
            L = gen.easy_lower(n, 200 + i)
            lids.append(T.trsm_server_register_L(srv, torch.from_numpy(L).cuda().data_ptr(), n, n))
            Ls.append(L)
        torch.cuda.synchronize()
        g = gen.rng(9)
        reqs = []
        for r in range(24):
            f = int(g.integers(0, len(ns)))
            k = int(gen.log_uniform_int(g, 1, 200))
            B = gen.rhs(ns[f], k, 900 + r)
            reqs.append(dict(f=f, k=k, B=B, Bd=torch.from_numpy(B).cuda(),
                             Xd=torch.full((ns[f], k), float("nan"), dtype=torch.float64,
                                           device="cuda")))
        torch.cuda.synchronize()
        lone = []
        for q in reqs:
            t = submit(T, srv, lids[q["f"]], q)
            assert wait_all(T, srv, [t])[t][0] == T.REQ_DONE
            lone.append(q["Xd"].cpu().numpy().copy())
            q["Xd"].fill_(float("nan"))
        torch.cuda.synchronize()
        errors = []
        extra = {}

        def submitter(part):
            try:
                mine = [q for i, q in enumerate(reqs) if i % 4 == part]
                ts = [submit(T, srv, lids[q["f"]], q) for q in mine]
                res = wait_all(T, srv, ts)
                assert all(res[t][0] == T.REQ_DONE for t in ts)
            except Exception as e:   # reported below
                errors.append(e)

        def registrar():
            try:
                L = gen.easy_lower(512, 777)
                Ld = torch.from_numpy(L).cuda()
                extra["lid"] = T.trsm_server_register_L(srv, Ld.data_ptr(), 512, 512)
                extra["L"] = L
            except Exception as e:
                errors.append(e)

        th = [threading.Thread(target=submitter, args=(p,)) for p in range(4)]
        th.append(threading.Thread(target=registrar))
        for x in th:
            x.start()
        for x in th:
            x.join()
        assert not errors, errors
        for q, X in zip(reqs, lone):
            Xc = q["Xd"].cpu().numpy()
            assert np.array_equal(Xc, X)
            assert oracle.rel_fro_err(Xc, oracle.trsm(Ls[q["f"]], q["B"])) <= 1e-12
        # the factor registered during the run serves correctly afterwards
        B = gen.rhs(512, 17, 5)
        Bd = torch.from_numpy(B).cuda()
        Xd = torch.empty_like(Bd)
        t = T.trsm_serve_submit(srv, extra["lid"], Bd.data_ptr(), 17, 17, Xd.data_ptr(), 17)
        assert wait_all(T, srv, [t])[t][0] == T.REQ_DONE
        assert oracle.rel_fro_err(Xd.cpu().numpy(), oracle.trsm(extra["L"], B)) <= 1e-12
        stats = T.trsm_server_stats(srv)
        assert stats.failed == 0 and stats.completed == 2 * len(reqs) + 1
    finally:
        T.trsm_server_destroy(srv)


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_ill_conditioned_factor_is_backward_stable(torch, T, precision):
    """cond(L) ~ 1e6: each request stops by its own test with a backward
    stable X, within the conditioning's reach of the oracle's X."""
    srv = T.trsm_server_create(2 << 30, 16)
    try:
        n = 900
        Lh = gen.hard_lower(n, 31, upper=np.nan, ratio=1e-12)
        lid = T.trsm_server_register_L(srv, torch.from_numpy(Lh).cuda().data_ptr(), n, n,
                                       precision)
        torch.cuda.synchronize()
        reqs = []
        for r, k in enumerate([1, 7, 64, 130]):
            B = gen.rhs(n, k, 40 + r)
            reqs.append(dict(k=k, B=B, Bd=torch.from_numpy(B).cuda(),
                             Xd=torch.full((n, k), float("nan"), dtype=torch.float64,
                                           device="cuda")))
        torch.cuda.synchronize()
        ts = [submit(T, srv, lid, q) for q in reqs]
        res = wait_all(T, srv, ts)
        for q, t in zip(reqs, ts):
            st, status, info = res[t]
            assert st == T.REQ_DONE and status == T.OK and info.converged == 1
            X = q["Xd"].cpu().numpy()
            berr = oracle.backward_err(Lh, X, q["B"])
            err = oracle.rel_fro_err(X, oracle.trsm(Lh, q["B"]))
            print(f"{precision} cond~1e6 k={q['k']}: {info.iterations} corrections, "
                  f"berr {berr:.1e} (server {info.backward_error:.1e}), "
                  f"unrefined {info.unrefined_error:.1e}, rel err vs oracle {err:.1e}", flush=True)
            assert berr <= 4 * np.sqrt(n) * U
            assert err <= 1e-8
    finally:
        T.trsm_server_destroy(srv)


def test_tolerance_below_the_residual_floor_stops_on_corrections(torch, T):
    """With a backward-error tolerance no residual meets, requests stop when
    the corrections stop mattering (two or more corrections), still OK."""
    srv = T.trsm_server_create(1 << 30, 8, 0, 1e-30)
    try:
        n = 700
        L = gen.easy_lower(n, 12, upper=np.nan)
        lid = T.trsm_server_register_L(srv, torch.from_numpy(L).cuda().data_ptr(), n, n)
        for r, k in enumerate([1, 40]):
            B = gen.rhs(n, k, 70 + r)
            Bd = torch.from_numpy(B).cuda()
            Xd = torch.full_like(Bd, float("nan"))
            torch.cuda.synchronize()
            t = T.trsm_serve_submit(srv, lid, Bd.data_ptr(), k, k, Xd.data_ptr(), k)
            st, status, info = wait_all(T, srv, [t])[t]
            print(f"k={k}: {info.iterations} corrections, last correction {info.correction:.1e}, "
                  f"berr {info.backward_error:.1e}", flush=True)
            assert st == T.REQ_DONE and status == T.OK and info.converged == 1
            assert info.iterations >= 2 and info.correction <= 1e-13
            assert oracle.rel_fro_err(Xd.cpu().numpy(), oracle.trsm(L, B)) <= 1e-12
    finally:
        T.trsm_server_destroy(srv)


def test_correction_cap_returns_not_converged(torch, T):
    """With one correction allowed and a tolerance nothing meets, every
    request ends DONE with TRSM_ENOTCONVERGED, X holding its last iterate
    (one correction: still accurate to about 1e-12 on this factor)."""
    srv = T.trsm_server_create(1 << 30, 8, 0, 1e-300, 1)
    try:
        n, k = 500, 20
        L = gen.easy_lower(n, 3, upper=np.nan)
        lid = T.trsm_server_register_L(srv, torch.from_numpy(L).cuda().data_ptr(), n, n)
        B = gen.rhs(n, k, 4)
        Bd = torch.from_numpy(B).cuda()
        Xd = torch.full_like(Bd, float("nan"))
        torch.cuda.synchronize()
        t = T.trsm_serve_submit(srv, lid, Bd.data_ptr(), k, k, Xd.data_ptr(), k)
        st, status, info = wait_all(T, srv, [t])[t]
        assert st == T.REQ_DONE and status == T.ENOTCONVERGED
        assert info.converged == 0 and info.iterations == 1
        assert oracle.rel_fro_err(Xd.cpu().numpy(), oracle.trsm(L, B)) <= 1e-9
        stats = T.trsm_server_stats(srv)
        assert stats.unconverged == 1 and stats.completed == 1 and stats.failed == 0
    finally:
        T.trsm_server_destroy(srv)


def test_zero_rhs_and_tiny_and_huge_scales(torch, T):
    """B = 0 converges at once to X = 0; right-hand sides scaled by 2^-600
    and 2^+600 (outside binary32's range) are solved through the per-pass
    power-of-two scaling, to the same relative accuracy."""
    srv = T.trsm_server_create(1 << 30, 8)
    try:
        n, k = 300, 9
        L = gen.easy_lower(n, 8, upper=np.nan)
        lid = T.trsm_server_register_L(srv, torch.from_numpy(L).cuda().data_ptr(), n, n)
        B0 = gen.rhs(n, k, 9)
        ref = oracle.trsm(L, B0)
        for scale in [0.0, 2.0 ** -600, 2.0 ** 600, 1.0]:
            B = B0 * scale
            Bd = torch.from_numpy(B).cuda()
            Xd = torch.full_like(Bd, float("nan"))
            torch.cuda.synchronize()
            t = T.trsm_serve_submit(srv, lid, Bd.data_ptr(), k, k, Xd.data_ptr(), k)
            st, status, info = wait_all(T, srv, [t])[t]
            assert st == T.REQ_DONE and status == T.OK and info.converged == 1
            X = Xd.cpu().numpy()
            if scale == 0.0:
                assert np.all(X == 0.0)
            else:
                assert oracle.rel_fro_err(X / scale, ref) <= 1e-12
    finally:
        T.trsm_server_destroy(srv)


def test_served_factors_at_serving_sizes(torch, T):
    """Factors of the serving workload's largest sizes (n = 2048 and 4076,
    each inverted whole: n0 = 4096), triangular and Cholesky, binary32 and
    binary64 sweeps, against the oracle."""
    srv = T.trsm_server_create(8 << 30, 16)
    try:
        spec = [(4076, False, "f32"), (2048, False, "f32"), (4076, False, "f64"),
                (2048, True, "f32")]
        Ls, lids = [], []
        for i, (n, chol, prec) in enumerate(spec):
            L = gen.chol_lower(n, 60 + i, upper=np.nan) if chol else \
                gen.easy_lower(n, 60 + i, upper=np.nan)
            Ld = torch.from_numpy(L).cuda()
            reg = T.trsm_server_register_chol if chol else T.trsm_server_register_L
            lids.append(reg(srv, Ld.data_ptr(), n, n, prec))
            Ls.append(L)
            del Ld
        torch.cuda.synchronize()
        reqs = []
        for r, (f, k) in enumerate([(0, 1), (0, 64), (1, 37), (2, 16), (3, 8), (1, 512)]):
            B = gen.rhs(spec[f][0], k, 90 + r)
            reqs.append(dict(f=f, k=k, B=B, Bd=torch.from_numpy(B).cuda(),
                             Xd=torch.full((spec[f][0], k), float("nan"), dtype=torch.float64,
                                           device="cuda")))
        torch.cuda.synchronize()
        ts = [submit(T, srv, lids[q["f"]], q) for q in reqs]
        res = wait_all(T, srv, ts)
        for q, t in zip(reqs, ts):
            st, status, info = res[t]
            assert st == T.REQ_DONE and status == T.OK and info.converged == 1
            n, chol, prec = spec[q["f"]]
            L = Ls[q["f"]]
            kc = min(q["k"], 64)   # the oracle on the first columns (columns are independent)
            ref = oracle.trsm(L, q["B"][:, :kc])
            if chol:
                ref = oracle.trsm_t(L, ref)
            X = q["Xd"].cpu().numpy()[:, :kc]
            err = oracle.rel_fro_err(X, ref)
            print(f"{prec} {'cholesky' if chol else 'triangular'} n={n} k={q['k']}: "
                  f"rel err {err:.2e}, {info.iterations} corrections", flush=True)
            assert err <= 1e-12
    finally:
        T.trsm_server_destroy(srv)


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_tiny_factors_and_narrow_right_hand_sides(torch, T, precision):
    # rows and columns below the padding granule (n = 1, 3, 5; k = 1, 2, 3,
    # 5): the grouped loads, conversions and norm reductions skip the padded
    # rows and columns of every internal buffer; triangular and Cholesky
    # factors share the batches
    srv = T.trsm_server_create(1 << 30, 32, 0)
    try:
        spec = [(1, False), (3, True), (5, False), (5, True), (67, True), (130, False)]
        Ls, lids = [], []
        for i, (n, chol) in enumerate(spec):
            L = gen.chol_lower(n, 700 + i, upper=np.nan) if chol else \
                gen.easy_lower(n, 700 + i, upper=np.nan)
            Ld = torch.from_numpy(L).cuda()
            reg = T.trsm_server_register_chol if chol else T.trsm_server_register_L
            lids.append(reg(srv, Ld.data_ptr(), n, n, precision))
            Ls.append(L)
            del Ld
        torch.cuda.synchronize()
        reqs = []
        for f in range(len(spec)):
            for j, k in enumerate([1, 2, 3, 5, 257]):
                B = gen.rhs(spec[f][0], k, 900 + 10 * f + j)
                Bd = torch.from_numpy(B).cuda()
                Xd = torch.full_like(Bd, float("nan"))
                reqs.append(dict(f=f, k=k, B=B, Bd=Bd, Xd=Xd))
        torch.cuda.synchronize()
        tickets = [submit(T, srv, lids[q["f"]], q) for q in reqs]
        res = wait_all(T, srv, tickets)
        mix = []
        for q, t in zip(reqs, tickets):
            st, status, info = res[t]
            assert st == T.REQ_DONE and status == T.OK
            X = q["Xd"].cpu().numpy()
            n, chol = spec[q["f"]]
            L = Ls[q["f"]]
            ref = oracle.trsm_t(L, oracle.trsm(L, q["B"])) if chol else oracle.trsm(L, q["B"])
            err = oracle.rel_fro_err(X, ref)
            print(f"{'cholesky' if chol else 'triangular'} n={n} k={q['k']}: "
                  f"rel err {err:.2e}, {info.iterations} corrections", flush=True)
            assert err <= 1e-12
            if chol:
                assert info.converged == 1
            else:
                check_info(info, n, precision)
            mix.append((X.copy(), info_tuple(info)))
        for q, (X, inf) in list(zip(reqs, mix))[::4]:
            q["Xd"].fill_(float("nan"))
            torch.cuda.synchronize()
            t = submit(T, srv, lids[q["f"]], q)
            st, status, info = wait_all(T, srv, [t])[t]
            assert st == T.REQ_DONE and status == T.OK
            assert np.array_equal(q["Xd"].cpu().numpy(), X)
            assert info_tuple(info) == inf
    finally:
        T.trsm_server_destroy(srv)
