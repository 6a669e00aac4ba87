"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/trsm.h declares, validates arguments, and plans the
blocking (Sec. VIII rule reported, n0 power of two, buffer sizes)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trsm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(trsm_[A-Za-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def T():
    from paper_1612_01855_amd import trsm
    return trsm


def test_header_declares_the_named_calls():
    names = declared_functions()
    for required in ["trsm_plan", "trsm_invert_diag", "trsm_solve"]:
        assert required in names


def test_library_exports_every_declared_symbol(T):
    lib = ctypes.CDLL(T.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []
    assert set(T.EXPORTS) <= set(declared_functions())


def test_status_strings(T):
    assert T.status_string(T.OK) == "TRSM_OK"
    assert T.status_string(T.ESINGULAR) == "TRSM_ESINGULAR"
    assert T.status_string(99) == "TRSM_UNKNOWN"


@pytest.mark.parametrize("args", [(-1, 4, 0, 0, 0), (4, -1, 0, 0, 0), (8, 8, 9, 0, 0),
                                  (8, 8, 0, 3, 0), (8, 8, 0, -2, 0), (8, 8, 0, 0, 0x80), (8, 8, 0, 0, 0x40),
                                  (8, 8, 2, 0, 2),
                                  # beyond the addressable sizes: n k > 2^31 - 1, n > 2^30
                                  (65536, 32769, 0, 0, 0), ((1 << 30) + 1, 1, 0, 0, 0),
                                  (1, (1 << 30) + 1, 0, 0, 0)])
def test_plan_rejects_bad_arguments(T, args):
    with pytest.raises(T.TrsmError) as e:
        T.trsm_plan(*args)
    assert e.value.status == T.EINVAL


def test_plan_null_out_pointer(T):
    lib = T._lib
    assert lib.trsm_plan(4, 4, 0, 0, 0, None) == T.EINVAL
    assert lib.trsm_plan_get_info(None, None) == T.EINVAL
    assert lib.trsm_plan_destroy(None) == T.OK


@pytest.mark.parametrize("n,k,expect", [(16384, 16384, 16384), (16384, 128, 431),
                                        (16384, 2048, 3444), (16384, 32768, 16384),
                                        (256, 64, 128), (4096, 1024, 2048)])
def test_paper_rule_reported(T, n, k, expect):
    # Sec. VIII at p = 1: n < 4k -> n0 = n; n > 4k -> (n k^3)^(1/4); n = 4k -> min(sqrt(nk), n)
    p = T.trsm_plan(n, k, T.F64, 0, 0)
    try:
        assert T.trsm_plan_get_info(p).n0_paper_rule == expect
    finally:
        T.trsm_plan_destroy(p)


@pytest.mark.parametrize("n,k,n0", [(256, 64, 32), (1000, 7, 0), (1, 1, 0), (0, 5, 0),
                                    (7, 0, 4), (300, 20, 1024), (8192, 8192, 0),
                                    (65536, 32767, 0)])   # the largest n k a plan accepts
def test_plan_layout(T, n, k, n0):
    p = T.trsm_plan(n, k, T.F64, n0, 0)
    try:
        i = T.trsm_plan_get_info(p)
        assert i.n0 >= 1 and (i.n0 & (i.n0 - 1)) == 0
        if n0:
            assert i.n0 == min(n0, 1 << max(n - 1, 0).bit_length())
        assert i.m == (-(-n // i.n0) if n else 0)
        assert i.leaf == min(i.n0, 64)
        assert i.linv_bytes >= i.m * i.n0 * i.n0 * 8
        assert i.workspace_bytes >= n * k * 8
        assert i.solve_flops == float(n) * n * k
    finally:
        T.trsm_plan_destroy(p)


def test_fp8_plan_is_a_mixed_plan(T):
    p = T.trsm_plan(300, 20, T.MIXED_FP8, 64, 0)
    try:
        i = T.trsm_plan_get_info(p)
        assert i.precision == T.MIXED_FP8 and i.n0 == 64
        assert i.linv_bytes >= 5 * 64 * 64 * 12 + 300 * 300
    finally:
        T.trsm_plan_destroy(p)
    with pytest.raises(T.TrsmError):
        T.trsm_plan(300, 20, T.MIXED_FP8, 64, T.FLAG_RECURSIVE)


def test_mixed_plan_has_low_precision_copies(T):
    p64 = T.trsm_plan(512, 64, T.F64, 128, 0)
    pb = T.trsm_plan(512, 64, T.MIXED_BF16, 128, 0)
    try:
        a, b = T.trsm_plan_get_info(p64), T.trsm_plan_get_info(pb)
        assert b.linv_bytes >= a.linv_bytes + 4 * 512 * 128 + 2 * 512 * 512
        assert b.workspace_bytes > a.workspace_bytes
    finally:
        T.trsm_plan_destroy(p64)
        T.trsm_plan_destroy(pb)


def test_batch_autotune_validation_without_gpu(T):
    lib = T._lib
    out = T.BatchTuneResult()
    n, _ = T._i64_array([100, 200])
    k, _ = T._i64_array([3, 4])
    bad0, _ = T._i64_array([100, 0])
    big, _ = T._i64_array([100, 70000])
    assert lib.trsm_batch_autotune(0, n, k, T.F64, 2, ctypes.byref(out)) == T.EINVAL
    assert lib.trsm_batch_autotune(2, None, k, T.F64, 2, ctypes.byref(out)) == T.EINVAL
    assert lib.trsm_batch_autotune(2, n, None, T.F64, 2, ctypes.byref(out)) == T.EINVAL
    assert lib.trsm_batch_autotune(2, n, k, T.F64, 0, ctypes.byref(out)) == T.EINVAL
    assert lib.trsm_batch_autotune(2, n, k, T.F64, 2, None) == T.EINVAL
    assert lib.trsm_batch_autotune(2, n, k, T.MIXED_F16, 2, ctypes.byref(out)) == T.EINVAL
    assert lib.trsm_batch_autotune(2, bad0, k, T.F64, 2, ctypes.byref(out)) == T.EINVAL
    assert lib.trsm_batch_autotune(2, big, k, T.F64, 2, ctypes.byref(out)) == T.EINVAL
    n0 = ctypes.c_int64(-1)
    assert lib.trsm_batch_autotune_lookup(2, n, k, T.F64, None) == T.EINVAL
    assert lib.trsm_batch_autotune_lookup(0, n, k, T.F64, ctypes.byref(n0)) == T.EINVAL
    T.trsm_autotune_clear()
    assert lib.trsm_batch_autotune_lookup(2, n, k, T.F64, ctypes.byref(n0)) == T.OK
    assert n0.value == 0


def test_plan_tolerance_validation(T):
    lib = T._lib
    assert lib.trsm_plan_set_tolerance(None, 1e-12) == T.EINVAL
    p = T.trsm_plan(512, 64, T.MIXED_F16, 128, 0)
    try:
        for bad in (-1e-12, 1.0, 2.0, float("nan"), float("inf")):
            assert lib.trsm_plan_set_tolerance(p, bad) == T.EINVAL
        for good in (0.0, 1e-12, 0.5):
            assert lib.trsm_plan_set_tolerance(p, good) == T.OK
    finally:
        T.trsm_plan_destroy(p)
    # binary64 plans keep the value and ignore it
    p = T.trsm_plan(64, 8, T.F64, 16, 0)
    try:
        assert lib.trsm_plan_set_tolerance(p, 1e-12) == T.OK
    finally:
        T.trsm_plan_destroy(p)


def test_solve_argument_validation_without_gpu(T):
    p = T.trsm_plan(64, 8, T.F64, 16, 0)
    try:
        lib = T._lib
        fake = 1 << 20      # never dereferenced: validation fails first
        # null L
        assert lib.trsm_solve(p, None, 64, fake, fake, 8, fake + 4096, 8, fake, None, None) == T.EINVAL
        # ldl < n
        assert lib.trsm_solve(p, fake, 63, fake, fake, 8, fake + 4096, 8, fake, None, None) == T.EINVAL
        # ldb < k
        assert lib.trsm_solve(p, fake, 64, fake, fake, 7, fake + 4096, 8, fake, None, None) == T.EINVAL
        # partial overlap of B and X
        assert lib.trsm_solve(p, fake, 64, fake, fake, 8, fake + 8, 8, fake, None, None) == T.EINVAL
        # misaligned workspace
        assert lib.trsm_solve(p, fake, 64, fake, fake, 8, fake + 65536, 8, fake + 8, None, None) == T.EINVAL
        # null Linv / L for invert
        assert lib.trsm_invert_diag(p, None, 64, fake, None) == T.EINVAL
        assert lib.trsm_invert_diag(p, fake, 10, fake, None) == T.EINVAL
    finally:
        T.trsm_plan_destroy(p)


def test_residual_validation_without_gpu(T):
    lib = T._lib
    norms = (ctypes.c_double * 3)()
    fake = 1 << 20
    assert lib.trsm_residual(4, 4, fake, 4, fake + 4096, 4, fake + 8192, 4, fake + 8192, 4,
                             fake, norms, None) == T.EINVAL   # R overlaps B
    assert lib.trsm_residual(4, 4, fake, 3, fake + 4096, 4, fake + 8192, 4, fake + 16384, 4,
                             fake, norms, None) == T.EINVAL   # ldl < n
    assert lib.trsm_residual(0, 4, None, 0, None, 4, None, 4, None, 4, None, norms, None) == T.OK


def test_batch_create_validation_and_workspace(T):
    fake = 1 << 24
    good = T.BatchItem(300, 7, fake, 300, fake, fake + (1 << 22), 7, fake + (1 << 23), 7)
    b = T.trsm_batch_create([good], T.F64, 128)
    try:
        ws = T.trsm_batch_workspace_bytes(b)
        assert ws >= 300 * 7 * 8          # running right-hand side
    finally:
        T.trsm_batch_destroy(b)
    bad_ld = T.BatchItem(300, 7, fake, 299, fake, fake + (1 << 22), 7, fake + (1 << 23), 7)
    overlap = T.BatchItem(300, 7, fake, 300, fake, fake + (1 << 22), 7, fake + (1 << 22) + 8, 7)
    misaligned = T.BatchItem(300, 7, fake, 300, fake + 8, fake + (1 << 22), 7, fake + (1 << 23), 7)
    for item in (bad_ld, overlap, misaligned):
        with pytest.raises(T.TrsmError) as e:
            T.trsm_batch_create([item], T.F64, 128)
        assert e.value.status == T.EINVAL
    with pytest.raises(T.TrsmError):
        T.trsm_batch_create([good], T.MIXED_BF16, 128)   # plain precisions only
    with pytest.raises(T.TrsmError):
        T.trsm_batch_create([good], T.F64, 96)            # n0 must be a power of two
    empty = T.trsm_batch_create([], T.F32, 64)
    T.trsm_batch_run(empty, 0, 0, False)                  # nothing to do: no device work
    T.trsm_batch_destroy(empty)


def test_server_argument_validation_without_gpu(T):
    lib = T._lib
    h = ctypes.c_void_p()
    assert lib.trsm_server_create(1 << 30, 0, ctypes.byref(h)) == T.EINVAL   # no slots
    assert lib.trsm_server_create(1 << 10, 8, ctypes.byref(h)) == T.EINVAL   # tiny budget
    assert lib.trsm_server_create(1 << 30, 8, None) == T.EINVAL
    bad = [T.ServerOptions(96, 0.0, 0, 0),      # n0 not a power of two
           T.ServerOptions(-64, 0.0, 0, 0),
           T.ServerOptions(0, -1.0, 0, 0),      # negative tolerance
           T.ServerOptions(0, float("nan"), 0, 0),
           T.ServerOptions(0, 0.0, -1, 0),      # correction cap out of range
           T.ServerOptions(0, 0.0, 51, 0),
           T.ServerOptions(0, 0.0, 0, 1)]       # reserved field set
    for o in bad:
        assert lib.trsm_server_create_ex(1 << 30, 8, ctypes.byref(o), ctypes.byref(h)) == T.EINVAL
        assert h.value is None
    assert lib.trsm_server_create_ex(1 << 30, 8, None, ctypes.byref(h)) == T.EINVAL
    st = ctypes.c_int()
    assert lib.trsm_serve_poll(None, 1, ctypes.byref(st), None) == T.EINVAL
    info = T.Info()
    assert lib.trsm_serve_poll(None, 1, ctypes.byref(st), ctypes.byref(info)) == T.EINVAL
    lid = ctypes.c_int32()
    assert lib.trsm_server_register_L(None, None, 10, 10, T.F32, ctypes.byref(lid)) == T.EINVAL
    assert lib.trsm_server_register_chol(None, None, 10, 10, T.F64, ctypes.byref(lid)) == T.EINVAL
    t = ctypes.c_uint64()
    assert lib.trsm_serve_submit(None, 0, None, 1, 1, None, 1, ctypes.byref(t)) == T.EINVAL
    assert lib.trsm_server_stats(None, None) == T.EINVAL
    assert lib.trsm_server_reset_stats(None) == T.EINVAL
    assert lib.trsm_server_destroy(None) == T.OK


def test_autotune_table_without_gpu(T):
    T.trsm_autotune_clear()
    assert T.trsm_autotune_lookup(1000, 64, T.F64) == (0, 0)
    lib = T._lib
    r = T.TuneResult()
    for args in [(0, 64, T.F64, 3), (100, 0, T.F64, 3), (100, 64, T.F64, 0),
                 (100, 64, T.MIXED_BF16, 3)]:
        assert lib.trsm_autotune(*args, None, ctypes.byref(r)) == T.EINVAL
    assert lib.trsm_autotune(100, 64, T.F64, 3, None, None) == T.EINVAL
    # the large-tile policy is a valid plan flag
    p = T.trsm_plan(300, 20, T.F64, 64, T.FLAG_LARGE_TILES)
    assert T.trsm_plan_get_info(p).flags == T.FLAG_LARGE_TILES
    T.trsm_plan_destroy(p)


def test_transposed_plans(T):
    p0 = T.trsm_plan(300, 20, T.F64, 64, 0)
    p1 = T.trsm_plan(300, 20, T.F64, 64, T.FLAG_TRANSPOSE)
    try:
        a, b = T.trsm_plan_get_info(p0), T.trsm_plan_get_info(p1)
        # L^T (300 x 300 with rows of 300) and the transposed blocks are kept too
        assert b.linv_bytes >= a.linv_bytes + 300 * 300 * 8 + 5 * 64 * 64 * 8
        assert b.workspace_bytes == a.workspace_bytes
    finally:
        T.trsm_plan_destroy(p0)
        T.trsm_plan_destroy(p1)
    for prec, flags in [(T.MIXED_BF16, T.FLAG_TRANSPOSE),
                        (T.F64, T.FLAG_TRANSPOSE | T.FLAG_RECURSIVE),
                        (T.F64, T.FLAG_TRANSPOSE | T.FLAG_LOOKAHEAD)]:
        with pytest.raises(T.TrsmError):
            T.trsm_plan(300, 20, prec, 64, flags)


def test_upper_plans(T):
    p0 = T.trsm_plan(300, 20, T.F64, 64, 0)
    p1 = T.trsm_plan(300, 20, T.F64, 64, T.FLAG_UPPER)
    p2 = T.trsm_plan(300, 20, T.F32, 64, T.FLAG_UPPER)
    try:
        a, b, c = (T.trsm_plan_get_info(p) for p in (p0, p1, p2))
        # U is read in place: only the inverses of its five diagonal blocks are added
        assert b.linv_bytes >= a.linv_bytes + 5 * 64 * 64 * 8
        assert b.linv_bytes < a.linv_bytes + 300 * 300 * 8
        assert b.workspace_bytes == a.workspace_bytes
        assert c.linv_bytes > 0 and b.flags & T.FLAG_UPPER
    finally:
        for p in (p0, p1, p2):
            T.trsm_plan_destroy(p)
    for prec, flags in [(T.MIXED_BF16, T.FLAG_UPPER), (T.MIXED_FP8, T.FLAG_UPPER),
                        (T.F64, T.FLAG_UPPER | T.FLAG_TRANSPOSE),
                        (T.F64, T.FLAG_UPPER | T.FLAG_RECURSIVE),
                        (T.F64, T.FLAG_UPPER | T.FLAG_LOOKAHEAD)]:
        with pytest.raises(T.TrsmError):
            T.trsm_plan(300, 20, prec, 64, flags)


def test_cholesky_sizes_and_validation_without_gpu(T):
    # default block: 512 from n = 12288 on, 256 below, at most pow2 >= max(n, 64)
    assert T.trsm_chol_sizes(10)[0] == 64
    assert T.trsm_chol_sizes(100)[0] == 128
    assert T.trsm_chol_sizes(4096)[0] == 128
    assert T.trsm_chol_sizes(6144)[0] == 256
    assert T.trsm_lu_sizes(4096)[0] == 128
    assert T.trsm_chol_sizes(8192)[0] == 256
    assert T.trsm_chol_sizes(16384)[0] == 512
    nb, lb, wb = T.trsm_chol_sizes(1000, 128)
    m = (1000 + 127) // 128
    assert nb == 128 and lb >= m * 128 * 128 * 8 and lb % 256 == 0
    # status word + nb^2 temp + two (n - nb) x nb panels + split-K scratch
    assert wb >= 256 + 128 * 128 * 8 + 2 * (1000 - 128) * 128 * 8
    # the Linv layout is a TRSM_F64 plan's with n0 = nb
    p = T.trsm_plan(1000, 8, T.F64, 128, 0)
    try:
        assert T.trsm_plan_get_info(p).linv_bytes == lb
    finally:
        T.trsm_plan_destroy(p)
    for bad_nb in (32, 96, 8192, -1):
        with pytest.raises(T.TrsmError):
            T.trsm_chol_sizes(100, bad_nb)
    with pytest.raises(T.TrsmError):
        T.trsm_chol_sizes(-1)
    with pytest.raises(T.TrsmError):
        T.trsm_chol_sizes((1 << 20) + 1)
    lib = T._lib
    fake = 1 << 20
    # null A / Linv / workspace, lda < n, misaligned workspace or Linv
    assert lib.trsm_chol_factor(64, None, 64, 0, fake, fake, None) == T.EINVAL
    assert lib.trsm_chol_factor(64, fake, 64, 0, None, fake, None) == T.EINVAL
    assert lib.trsm_chol_factor(64, fake, 64, 0, fake, None, None) == T.EINVAL
    assert lib.trsm_chol_factor(64, fake, 63, 0, fake, fake, None) == T.EINVAL
    assert lib.trsm_chol_factor(64, fake, 64, 0, fake, fake + 8, None) == T.EINVAL
    assert lib.trsm_chol_factor(64, fake, 64, 0, fake + 8, fake, None) == T.EINVAL
    assert lib.trsm_chol_factor(64, fake, 64, 48, fake, fake, None) == T.EINVAL
    assert lib.trsm_chol_check(None, None, None) == T.EINVAL


def test_lu_sizes_and_validation_without_gpu(T):
    nb, lb, wb = T.trsm_lu_sizes(1000, 128)
    cb = T.trsm_chol_sizes(1000, 128)
    assert nb == 128 and lb == cb[1]
    # the Cholesky workspace plus two nb x (n - nb) panels of U
    assert wb >= cb[2] + 2 * (1000 - 128) * 128 * 8
    for bad_nb in (32, 96, 8192):
        with pytest.raises(T.TrsmError):
            T.trsm_lu_sizes(100, bad_nb)
    # a block beyond the next power of two >= n is cut to it (a plan's n0 cap),
    # and the inverse buffer is a TRSM_F64 plan's Linv buffer for that n0
    nb, lb, _ = T.trsm_lu_sizes(100, 256)
    assert nb == 128
    p = T.trsm_plan(100, 5, T.F64, 128, 0)
    try:
        assert T.trsm_plan_get_info(p).linv_bytes == lb
    finally:
        T.trsm_plan_destroy(p)
    lib = T._lib
    fake = 1 << 20
    assert lib.trsm_lu_factor(64, None, 64, 0, fake, fake, fake, None) == T.EINVAL
    assert lib.trsm_lu_factor(64, fake, 64, 0, None, fake, fake, None) == T.EINVAL
    assert lib.trsm_lu_factor(64, fake, 64, 0, fake, None, fake, None) == T.EINVAL
    assert lib.trsm_lu_factor(64, fake, 63, 0, fake, fake, fake, None) == T.EINVAL
    assert lib.trsm_lu_factor(64, fake, 64, 0, fake, fake + 8, fake, None) == T.EINVAL
    assert lib.trsm_lu_factor(64, fake, 64, 0, fake, fake, fake + 8, None) == T.EINVAL


def test_binding_refuses_host_tensors_and_overlapping_rows(T):
    # a host tensor must never reach the library as a device pointer; the
    # binding refuses it (and wrong element types, overlapping rows) first
    import torch
    A = torch.zeros((8, 8), dtype=torch.float64)
    with pytest.raises(ValueError, match="CUDA"):
        T.Cholesky(8, 0, device="cpu").factor(A)
    with pytest.raises(ValueError, match="CUDA"):
        T.LU(8, 0, device="cpu").factor(A)
    with pytest.raises(ValueError, match="CUDA"):
        T._dev(A, torch.float64, "L")
    with pytest.raises(ValueError, match="overlap"):
        T._ld(torch.zeros(64, dtype=torch.float64).as_strided((8, 8), (1, 1)))
    assert T._ld(torch.zeros((5, 0))) == 1
    assert T._ld(torch.zeros((3, 7))[:, :4]) == 7


def test_pivoted_lu_sizes_and_validation_without_gpu(T):
    nbu, lb, wb = T.trsm_lu_piv_sizes(1000)
    assert nbu == 256 and lb == 4 * 256 * 256 * 8 and wb > 0
    assert T.trsm_lu_piv_sizes(20000)[0] == 512
    assert T.trsm_lu_piv_sizes(20)[0] == 32          # capped at pow2(n), at least one panel
    assert T.trsm_lu_piv_sizes(100, 512)[0] == 128
    lib = T._lib
    a, b, c = ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_size_t()
    for n, nb in [(0, 0), (-5, 0), (65537, 0), (100, 48), (100, 16), (100, -64)]:
        assert lib.trsm_lu_piv_sizes(n, nb, ctypes.byref(a), ctypes.byref(b),
                                     ctypes.byref(c)) == T.EINVAL
    # null or misaligned pointers are refused before any device work
    assert lib.trsm_lu_piv_factor(100, None, 100, 0, None, None, None, None) == T.EINVAL
    assert lib.trsm_lu_piv_factor(100, 256, 99, 0, 256, 256, 256, None) == T.EINVAL   # lda < n
    assert lib.trsm_lu_piv_factor(100, 256, 100, 0, 256, 256, 300, None) == T.EINVAL  # ws align
    st = ctypes.c_int()
    assert lib.trsm_lu_piv_check(None, ctypes.byref(st), None) == T.EINVAL
    assert lib.trsm_row_swaps(0, 5, None, None, 4, 4, None) == T.EINVAL
    assert lib.trsm_row_swaps(3, 2, None, None, 4, 4, None) == T.EINVAL
    assert lib.trsm_row_swaps(0, 0, None, None, 4, 4, None) == T.OK             # nothing to do


def test_product_path_is_independent_of_the_oracle():
    # the package and the library it builds name no part of the checker: no
    # import of `oracle`, no source that includes or links its files, and
    # the built library does not depend on the oracle's shared object
    pkg = os.path.join(ROOT, "paper_1612_01855_amd")
    for dirpath, _, files in os.walk(pkg):
        if "_build" in dirpath:
            continue
        for f in files:
            if not f.endswith((".py", ".hip", ".hpp", ".h")):
                continue
            text = open(os.path.join(dirpath, f)).read()
            assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
            assert "liboracle" not in text and "oracle.c" not in text, f
            assert not re.search(r'#include\s+"[^"]*oracle', text), f
    lib = os.path.join(pkg, "libtrsm.so")
    if os.path.exists(lib):
        assert b"liboracle" not in open(lib, "rb").read()


def test_binding_fails_loudly_without_the_library(tmp_path):
    # a copy of the package without libtrsm.so: importing the binding raises
    # (there is no fallback that could compute anything on the CPU)
    import shutil
    import subprocess
    import sys
    src = os.path.join(ROOT, "paper_1612_01855_amd")
    dst = tmp_path / "paper_1612_01855_amd"
    shutil.copytree(src, dst, ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__"))
    r = subprocess.run([sys.executable, "-c",
                        "import sys; sys.path.insert(0, sys.argv[1]); "
                        "from paper_1612_01855_amd import trsm", str(tmp_path)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "libtrsm.so is missing" in r.stderr
