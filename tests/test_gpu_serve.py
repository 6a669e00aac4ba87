"""GPU tests of the continuous-batching server: every request matches the
oracle on its own (L, B) (binary32 sweeps + one binary64 refinement step,
gate 1e-12), a request's result is bitwise the same alone and in a mix,
admission respects the HBM budget, and an impossible request fails cleanly."""
import time

import numpy as np
import pytest

import oracle
from paper_1612_01855_amd import inputs as gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a ROCm device"
    return _t


@pytest.fixture(scope="module")
def T():
    from paper_1612_01855_amd import trsm
    return trsm


def wait_all(T, srv, tickets, timeout=60.0):
    out = {}
    t0 = time.time()
    pending = set(tickets)
    while pending:
        for t in list(pending):
            st, status, lat = T.trsm_serve_poll(srv, t)
            if st in (T.REQ_DONE, T.REQ_ERROR):
                out[t] = (st, status, lat)
                pending.discard(t)
        assert time.time() - t0 < timeout, "server did not finish in time"
        time.sleep(0.001)
    return out


@pytest.mark.parametrize("n0", [128, 64, 4096])   # 64: persistent sweeps; 4096: full inverses
def test_server_requests_match_oracle_and_mix_independence(torch, T, n0):
    srv = T.trsm_server_create(2 << 30, 32, n0)
    try:
        ns = [64, 200, 777, 1300]
        Ls, lids = [], []
        for i, n in enumerate(ns):
            L = gen.easy_lower(n, 100 + i, upper=np.nan)
            Ld = torch.from_numpy(L).cuda()
            lids.append(T.trsm_server_register_L(srv, Ld.data_ptr(), n, n))
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
        tickets = [T.trsm_serve_submit(srv, lids[q["f"]], q["Bd"].data_ptr(), q["k"], q["k"],
                                       q["Xd"].data_ptr(), q["k"]) for q in reqs]
        res = wait_all(T, srv, tickets)
        mix = []
        for q, t in zip(reqs, tickets):
            st, status, lat = res[t]
            assert st == T.REQ_DONE and status == T.OK
            X = q["Xd"].cpu().numpy()
            err = oracle.rel_fro_err(X, oracle.trsm(Ls[q["f"]], q["B"]))
            print(f"request n={ns[q['f']]} k={q['k']}: rel err {err:.2e}, latency {lat:.0f} us",
                  flush=True)
            assert err <= 1e-12
            mix.append(X.copy())
        # the same requests one at a time give the same bits
        for q, X in zip(reqs[:6], mix[:6]):
            q["Xd"].fill_(float("nan"))
            torch.cuda.synchronize()
            t = T.trsm_serve_submit(srv, lids[q["f"]], q["Bd"].data_ptr(), q["k"], q["k"],
                                    q["Xd"].data_ptr(), q["k"])
            st, status, _ = wait_all(T, srv, [t])[t]
            assert st == T.REQ_DONE
            assert np.array_equal(q["Xd"].cpu().numpy(), X)
        stats = T.trsm_server_stats(srv)
        assert stats.completed == 22 and stats.failed == 0
        assert stats.p99_us >= stats.p50_us > 0
    finally:
        T.trsm_server_destroy(srv)


@pytest.mark.parametrize("n0", [128, 64])
def test_admission_respects_budget(torch, T, n0):
    n, k = 1024, 64
    # one factor (~12.6 MB) plus room for about two requests (~2 MB each)
    budget = 20 << 20
    srv = T.trsm_server_create(budget, 64, n0)
    try:
        L = gen.easy_lower(n, 7, upper=np.nan)
        Ld = torch.from_numpy(L).cuda()
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
            assert res[t][0] == T.REQ_DONE
            assert oracle.rel_fro_err(Xd.cpu().numpy(), oracle.trsm(L, B)) <= 1e-12
        stats = T.trsm_server_stats(srv)
        per_req = 32 * n * k
        assert stats.max_in_flight * per_req <= budget - stats.resident_bytes
        assert stats.max_in_flight >= 1
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


@pytest.mark.parametrize("n0", [128, 4096])
def test_cholesky_factors_mixed_with_triangular_ones(torch, T, n0):
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
            lids.append(reg(srv, Ld.data_ptr(), n, n))
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
        tickets = [T.trsm_serve_submit(srv, lids[q["f"]], q["Bd"].data_ptr(), q["k"], q["k"],
                                       q["Xd"].data_ptr(), q["k"]) for q in reqs]
        res = wait_all(T, srv, tickets)
        mix = []
        for q, t in zip(reqs, tickets):
            st, status, lat = res[t]
            assert st == T.REQ_DONE and status == T.OK
            L = Ls[q["f"]]
            ref = oracle.trsm_t(L, oracle.trsm(L, q["B"])) if spec[q["f"]][1] else \
                oracle.trsm(L, q["B"])
            X = q["Xd"].cpu().numpy()
            err = oracle.rel_fro_err(X, ref)
            print(f"{'cholesky' if spec[q['f']][1] else 'triangular'} n={spec[q['f']][0]} "
                  f"k={q['k']}: rel err {err:.2e}", flush=True)
            assert err <= 1e-12
            mix.append(X.copy())
        for q, X in zip(reqs[:5], mix[:5]):
            q["Xd"].fill_(float("nan"))
            torch.cuda.synchronize()
            t = T.trsm_serve_submit(srv, lids[q["f"]], q["Bd"].data_ptr(), q["k"], q["k"],
                                    q["Xd"].data_ptr(), q["k"])
            assert wait_all(T, srv, [t])[t][0] == T.REQ_DONE
            assert np.array_equal(q["Xd"].cpu().numpy(), X)
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
            t = T.trsm_serve_submit(srv, lids[q["f"]], q["Bd"].data_ptr(), q["k"], q["k"],
                                    q["Xd"].data_ptr(), q["k"])
            assert wait_all(T, srv, [t])[t][0] == T.REQ_DONE
            lone.append(q["Xd"].cpu().numpy().copy())
            q["Xd"].fill_(float("nan"))
        torch.cuda.synchronize()
        errors = []
        extra = {}

        def submitter(part):
            try:
                mine = [q for i, q in enumerate(reqs) if i % 4 == part]
                ts = [T.trsm_serve_submit(srv, lids[q["f"]], q["Bd"].data_ptr(), q["k"], q["k"],
                                          q["Xd"].data_ptr(), q["k"]) for q in mine]
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
