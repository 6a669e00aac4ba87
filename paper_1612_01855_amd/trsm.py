"""Thin ctypes binding of ``include/trsm.h`` (argument marshalling only).

Every function with a ``trsm_`` name forwards to the C entry point of the
same name in ``libtrsm.so``; all arithmetic happens in the library's HIP
kernels.  PyTorch is used only to own device memory and to name the stream:
tensors are passed as raw device pointers (``data_ptr()``) with their row
strides as leading dimensions.

The library must have been built (``python -m paper_1612_01855_amd.build``);
importing this module without it raises ``RuntimeError`` -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtrsm.so")

# trsm_status
OK, EINVAL, ESINGULAR, ENOMEM, EHIP, ENOTCONVERGED, EBUSY = range(7)
# trsm_precision
F64, F32, MIXED_BF16, MIXED_F16, MIXED_FP8 = range(5)
PRECISIONS = {"f64": F64, "f32": F32, "bf16": MIXED_BF16, "f16": MIXED_F16, "fp8": MIXED_FP8}
# plan flags
FLAG_NO_REFINE = 0x1
FLAG_RECURSIVE = 0x2
FLAG_LOOKAHEAD = 0x4
FLAG_LARGE_TILES = 0x8
FLAG_TRANSPOSE = 0x10
FLAG_UPPER = 0x20


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("k", ctypes.c_int64), ("n0", ctypes.c_int64),
                ("m", ctypes.c_int64), ("leaf", ctypes.c_int64),
                ("n0_paper_rule", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("linv_bytes", ctypes.c_size_t),
                ("workspace_bytes", ctypes.c_size_t), ("inv_flops", ctypes.c_double),
                ("solve_flops", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("backward_error", ctypes.c_double), ("correction", ctypes.c_double),
                ("unrefined_error", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int64), ("flags", ctypes.c_uint32), ("ms", ctypes.c_double),
                ("model_n0", ctypes.c_int64), ("model_ms", ctypes.c_double),
                ("candidates", ctypes.c_int32)]


class BatchTuneResult(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int64), ("ms", ctypes.c_double), ("default_n0", ctypes.c_int64),
                ("default_ms", ctypes.c_double), ("candidates", ctypes.c_int32)]


class BatchItem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("k", ctypes.c_int64), ("L", ctypes.c_void_p),
                ("ldl", ctypes.c_int64), ("Linv", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("ldb", ctypes.c_int64), ("X", ctypes.c_void_p), ("ldx", ctypes.c_int64)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("unconverged", ctypes.c_uint64), ("passes", ctypes.c_uint64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("flops_done", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("hbm_budget", ctypes.c_size_t),
                ("hbm_in_use", ctypes.c_size_t), ("resident_bytes", ctypes.c_size_t),
                ("queue_depth", ctypes.c_int32), ("in_flight", ctypes.c_int32),
                ("max_in_flight", ctypes.c_int32), ("factors", ctypes.c_int32)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int64), ("tolerance", ctypes.c_double),
                ("max_corrections", ctypes.c_int32), ("reserved", ctypes.c_int32)]


# trsm_req_state
REQ_PENDING, REQ_RUNNING, REQ_DONE, REQ_ERROR, REQ_UNKNOWN = range(5)

EXPORTS = ["trsm_status_string", "trsm_last_hip_error", "trsm_plan", "trsm_plan_get_info",
           "trsm_plan_destroy", "trsm_invert_diag", "trsm_plan_last_error", "trsm_solve",
           "trsm_solve_noalloc", "trsm_solve_noalloc_max_bytes",
           "trsm_residual_workspace_bytes", "trsm_residual", "trsm_plan_set_tolerance",
           "trsm_plan_set_timing",
           "trsm_plan_timing", "trsm_autotune", "trsm_autotune_lookup", "trsm_autotune_clear",
           "trsm_batch_autotune", "trsm_batch_autotune_lookup",
           "trsm_batch_create", "trsm_batch_workspace_bytes",
           "trsm_batch_run", "trsm_batch_check", "trsm_batch_destroy", "trsm_server_create",
           "trsm_server_create_ex", "trsm_server_register_L", "trsm_server_register_chol", "trsm_serve_submit", "trsm_serve_request_bytes",
           "trsm_serve_poll",
           "trsm_server_stats", "trsm_server_reset_stats", "trsm_server_destroy",
           "trsm_chol_sizes", "trsm_chol_factor", "trsm_chol_check",
           "trsm_lu_sizes", "trsm_lu_factor", "trsm_lu_check",
           "trsm_lu_piv_sizes", "trsm_lu_piv_factor", "trsm_lu_piv_check", "trsm_row_swaps"]


class TrsmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}"
                         + (f" (hip error {_lib.trsm_last_hip_error()})" if status == EHIP else ""))


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1612_01855_amd.build` (no fallback path exists)")
    # torch ships its own HIP runtime under the same soname as the one the
    # library links; loading torch first makes the library bind to that one,
    # so that one process never holds two HIP runtimes (device memory from
    # one is unknown to the other)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    i64, u32, vp, i32 = ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
    lib.trsm_status_string.argtypes = [i32]
    lib.trsm_status_string.restype = ctypes.c_char_p
    lib.trsm_last_hip_error.argtypes = []
    lib.trsm_last_hip_error.restype = i32
    lib.trsm_plan.argtypes = [i64, i64, i32, i64, u32, ctypes.POINTER(vp)]
    lib.trsm_plan.restype = i32
    lib.trsm_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.trsm_plan_get_info.restype = i32
    lib.trsm_plan_destroy.argtypes = [vp]
    lib.trsm_plan_destroy.restype = i32
    lib.trsm_invert_diag.argtypes = [vp, vp, i64, vp, vp]
    lib.trsm_invert_diag.restype = i32
    lib.trsm_plan_last_error.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    lib.trsm_plan_last_error.restype = i32
    lib.trsm_solve.argtypes = [vp, vp, i64, vp, vp, i64, vp, i64, vp, vp, ctypes.POINTER(Info)]
    lib.trsm_solve.restype = i32
    lib.trsm_solve_noalloc.argtypes = [vp, vp, i64, vp, vp, i64, vp, i64, vp, ctypes.POINTER(Info)]
    lib.trsm_solve_noalloc.restype = i32
    lib.trsm_solve_noalloc_max_bytes.argtypes = []
    lib.trsm_solve_noalloc_max_bytes.restype = ctypes.c_size_t
    lib.trsm_residual_workspace_bytes.argtypes = [i64, i64]
    lib.trsm_residual_workspace_bytes.restype = ctypes.c_size_t
    lib.trsm_residual.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp,
                                  ctypes.POINTER(ctypes.c_double), vp]
    lib.trsm_residual.restype = i32
    lib.trsm_plan_set_tolerance.argtypes = [vp, ctypes.c_double]
    lib.trsm_plan_set_tolerance.restype = i32
    lib.trsm_plan_set_timing.argtypes = [vp, i32]
    lib.trsm_plan_set_timing.restype = i32
    lib.trsm_plan_timing.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    lib.trsm_plan_timing.restype = i32
    lib.trsm_autotune.argtypes = [i64, i64, i32, ctypes.c_int32, vp, ctypes.POINTER(TuneResult)]
    lib.trsm_autotune.restype = i32
    lib.trsm_autotune_lookup.argtypes = [i64, i64, i32, ctypes.POINTER(i64), ctypes.POINTER(u32)]
    lib.trsm_autotune_lookup.restype = i32
    lib.trsm_batch_autotune.argtypes = [i32, ctypes.POINTER(i64), ctypes.POINTER(i64), i32,
                                        ctypes.c_int32, ctypes.POINTER(BatchTuneResult)]
    lib.trsm_batch_autotune.restype = i32
    lib.trsm_batch_autotune_lookup.argtypes = [i32, ctypes.POINTER(i64), ctypes.POINTER(i64), i32,
                                               ctypes.POINTER(i64)]
    lib.trsm_batch_autotune_lookup.restype = i32
    lib.trsm_autotune_clear.argtypes = []
    lib.trsm_autotune_clear.restype = i32
    lib.trsm_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(BatchItem), i32, i64,
                                      ctypes.POINTER(vp)]
    lib.trsm_batch_create.restype = i32
    lib.trsm_batch_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.trsm_batch_workspace_bytes.restype = i32
    lib.trsm_batch_run.argtypes = [vp, vp, vp, ctypes.c_int32]
    lib.trsm_batch_run.restype = i32
    lib.trsm_batch_check.argtypes = [vp, vp]
    lib.trsm_batch_check.restype = i32
    lib.trsm_batch_destroy.argtypes = [vp]
    lib.trsm_batch_destroy.restype = i32
    lib.trsm_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(vp)]
    lib.trsm_server_create.restype = i32
    lib.trsm_server_create_ex.argtypes = [ctypes.c_size_t, ctypes.c_int32,
                                          ctypes.POINTER(ServerOptions), ctypes.POINTER(vp)]
    lib.trsm_server_create_ex.restype = i32
    lib.trsm_server_register_L.argtypes = [vp, vp, i64, i64, i32, ctypes.POINTER(ctypes.c_int32)]
    lib.trsm_server_register_L.restype = i32
    lib.trsm_server_register_chol.argtypes = [vp, vp, i64, i64, i32,
                                              ctypes.POINTER(ctypes.c_int32)]
    lib.trsm_server_register_chol.restype = i32
    lib.trsm_serve_submit.argtypes = [vp, ctypes.c_int32, vp, i64, i64, vp, i64,
                                      ctypes.POINTER(ctypes.c_uint64)]
    lib.trsm_serve_submit.restype = i32
    lib.trsm_serve_request_bytes.argtypes = [vp, ctypes.c_int32, i64,
                                             ctypes.POINTER(ctypes.c_size_t)]
    lib.trsm_serve_request_bytes.restype = i32
    lib.trsm_serve_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32),
                                    ctypes.POINTER(Info)]
    lib.trsm_serve_poll.restype = i32
    lib.trsm_server_stats.argtypes = [vp, ctypes.POINTER(ServeStats)]
    lib.trsm_server_stats.restype = i32
    lib.trsm_server_reset_stats.argtypes = [vp]
    lib.trsm_server_reset_stats.restype = i32
    lib.trsm_server_destroy.argtypes = [vp]
    lib.trsm_server_destroy.restype = i32
    lib.trsm_chol_sizes.argtypes = [i64, i64, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.POINTER(ctypes.c_size_t)]
    lib.trsm_chol_sizes.restype = i32
    lib.trsm_chol_factor.argtypes = [i64, vp, i64, i64, vp, vp, vp]
    lib.trsm_chol_factor.restype = i32
    lib.trsm_chol_check.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    lib.trsm_chol_check.restype = i32
    lib.trsm_lu_sizes.argtypes = [i64, i64, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_size_t),
                                  ctypes.POINTER(ctypes.c_size_t)]
    lib.trsm_lu_sizes.restype = i32
    lib.trsm_lu_factor.argtypes = [i64, vp, i64, i64, vp, vp, vp, vp]
    lib.trsm_lu_factor.restype = i32
    lib.trsm_lu_check.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    lib.trsm_lu_check.restype = i32
    lib.trsm_lu_piv_sizes.argtypes = [i64, i64, ctypes.POINTER(i64),
                                      ctypes.POINTER(ctypes.c_size_t),
                                      ctypes.POINTER(ctypes.c_size_t)]
    lib.trsm_lu_piv_sizes.restype = i32
    lib.trsm_lu_piv_factor.argtypes = [i64, vp, i64, i64, vp, vp, vp, vp]
    lib.trsm_lu_piv_factor.restype = i32
    lib.trsm_lu_piv_check.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    lib.trsm_lu_piv_check.restype = i32
    lib.trsm_row_swaps.argtypes = [i64, i64, vp, vp, i64, i64, vp]
    lib.trsm_row_swaps.restype = i32
    return lib


_lib = _load()


def status_string(status: int) -> str:
    return _lib.trsm_status_string(int(status)).decode()


def _check(status: int, where: str):
    if status != OK:
        raise TrsmError(status, where)


# ---- raw entry points (same names as the C ABI) ------------------------------

def trsm_plan(n: int, k: int, precision: int = F64, n0: int = 0, flags: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(_lib.trsm_plan(n, k, precision, n0, flags, ctypes.byref(h)), "trsm_plan")
    return h.value


def trsm_plan_get_info(plan: int) -> PlanInfo:
    info = PlanInfo()
    _check(_lib.trsm_plan_get_info(plan, ctypes.byref(info)), "trsm_plan_get_info")
    return info


def trsm_plan_destroy(plan: int) -> None:
    _check(_lib.trsm_plan_destroy(plan), "trsm_plan_destroy")


def trsm_invert_diag(plan: int, L: int, ldl: int, Linv: int, stream: int = 0) -> None:
    _check(_lib.trsm_invert_diag(plan, L, ldl, Linv, stream), "trsm_invert_diag")


def trsm_plan_last_error(plan: int):
    st, idx = ctypes.c_int(), ctypes.c_int64()
    _check(_lib.trsm_plan_last_error(plan, ctypes.byref(st), ctypes.byref(idx)),
           "trsm_plan_last_error")
    return st.value, idx.value


def trsm_solve(plan: int, L: int, ldl: int, Linv: int, B: int, ldb: int, X: int, ldx: int,
               workspace: int, stream: int = 0, info: Optional[Info] = None) -> int:
    """Returns the raw status (TRSM_ENOTCONVERGED is not raised)."""
    st = _lib.trsm_solve(plan, L, ldl, Linv, B, ldb, X, ldx, workspace, stream,
                         ctypes.byref(info) if info is not None else None)
    if st not in (OK, ENOTCONVERGED):
        raise TrsmError(st, "trsm_solve")
    return st


def trsm_solve_noalloc(plan: int, L: int, ldl: int, Linv: int, B: int, ldb: int, X: int,
                       ldx: int, stream: int = 0, info: Optional[Info] = None) -> int:
    """The allocation-free solve; returns the raw status (no exception)."""
    return int(_lib.trsm_solve_noalloc(plan, L, ldl, Linv, B, ldb, X, ldx, stream,
                                       ctypes.byref(info) if info is not None else None))


def trsm_solve_noalloc_max_bytes() -> int:
    return int(_lib.trsm_solve_noalloc_max_bytes())


def trsm_residual_workspace_bytes(n: int, k: int) -> int:
    return int(_lib.trsm_residual_workspace_bytes(n, k))


def trsm_residual(n: int, k: int, L: int, ldl: int, X: int, ldx: int, B: int, ldb: int,
                  R: int, ldr: int, workspace: int, stream: int = 0):
    norms = (ctypes.c_double * 3)()
    _check(_lib.trsm_residual(n, k, L, ldl, X, ldx, B, ldb, R, ldr, workspace, norms, stream),
           "trsm_residual")
    return tuple(norms)


def trsm_plan_set_tolerance(plan: int, tol: float) -> None:
    _check(_lib.trsm_plan_set_tolerance(plan, float(tol)), "trsm_plan_set_tolerance")


def trsm_plan_set_timing(plan: int, enable: bool = True) -> None:
    _check(_lib.trsm_plan_set_timing(plan, 1 if enable else 0), "trsm_plan_set_timing")


def trsm_plan_timing(plan: int):
    """(launches, milliseconds, algorithmic flops) of the timed launches."""
    n, ms, fl = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(_lib.trsm_plan_timing(plan, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl)),
           "trsm_plan_timing")
    return n.value, ms.value, fl.value


def trsm_batch_create(items, precision: int = F64, n0: int = 128) -> int:
    arr = (BatchItem * max(len(items), 1))(*items)
    h = ctypes.c_void_p()
    _check(_lib.trsm_batch_create(len(items), arr, precision, n0, ctypes.byref(h)),
           "trsm_batch_create")
    return h.value


def trsm_batch_workspace_bytes(batch: int) -> int:
    v = ctypes.c_size_t()
    _check(_lib.trsm_batch_workspace_bytes(batch, ctypes.byref(v)), "trsm_batch_workspace_bytes")
    return v.value


def trsm_batch_run(batch: int, workspace: int, stream: int = 0, use_graph: bool = False) -> None:
    _check(_lib.trsm_batch_run(batch, workspace, stream, 1 if use_graph else 0), "trsm_batch_run")


def trsm_autotune(n: int, k: int, precision: int, reps: int = 3, stream: int = 0) -> TuneResult:
    r = TuneResult()
    _check(_lib.trsm_autotune(n, k, precision, reps, stream, ctypes.byref(r)), "trsm_autotune")
    return r


def _i64_array(vals):
    vals = [int(v) for v in vals]
    return (ctypes.c_int64 * max(len(vals), 1))(*vals), len(vals)


def trsm_batch_autotune(ns, ks, precision: int, reps: int = 3) -> BatchTuneResult:
    """Common block size of a batch of systems of sizes (ns[i], ks[i]),
    measured on the device (blocking)."""
    if len(ns) != len(ks):
        raise ValueError("ns and ks must have the same length")
    an, c = _i64_array(ns)
    ak, _ = _i64_array(ks)
    r = BatchTuneResult()
    _check(_lib.trsm_batch_autotune(c, an, ak, precision, reps, ctypes.byref(r)),
           "trsm_batch_autotune")
    return r


def trsm_batch_autotune_lookup(ns, ks, precision: int) -> int:
    """The recorded block size for a batch like this one, or 0."""
    if len(ns) != len(ks):
        raise ValueError("ns and ks must have the same length")
    an, c = _i64_array(ns)
    ak, _ = _i64_array(ks)
    n0 = ctypes.c_int64()
    _check(_lib.trsm_batch_autotune_lookup(c, an, ak, precision, ctypes.byref(n0)),
           "trsm_batch_autotune_lookup")
    return n0.value


def trsm_autotune_lookup(n: int, k: int, precision: int):
    """(n0, flags) recorded for this size class, or (0, 0)."""
    n0, fl = ctypes.c_int64(), ctypes.c_uint32()
    _check(_lib.trsm_autotune_lookup(n, k, precision, ctypes.byref(n0), ctypes.byref(fl)),
           "trsm_autotune_lookup")
    return n0.value, fl.value


def trsm_autotune_clear() -> None:
    _check(_lib.trsm_autotune_clear(), "trsm_autotune_clear")


def trsm_batch_check(batch: int, workspace: int) -> None:
    """Blocking: raises if a dependency wait of the persistent sweep gave up."""
    _check(_lib.trsm_batch_check(batch, workspace), "trsm_batch_check")


def trsm_batch_destroy(batch: int) -> None:
    _check(_lib.trsm_batch_destroy(batch), "trsm_batch_destroy")


def trsm_server_create(hbm_budget: int, max_slots: int = 64, n0: int = 0,
                       tolerance: float = 0.0, max_corrections: int = 0) -> int:
    """A server; n0, tolerance, max_corrections = 0 keep the library's defaults."""
    h = ctypes.c_void_p()
    if n0 or tolerance or max_corrections:
        opt = ServerOptions(n0, tolerance, max_corrections, 0)
        _check(_lib.trsm_server_create_ex(hbm_budget, max_slots, ctypes.byref(opt),
                                          ctypes.byref(h)), "trsm_server_create_ex")
    else:
        _check(_lib.trsm_server_create(hbm_budget, max_slots, ctypes.byref(h)),
               "trsm_server_create")
    return h.value


def trsm_server_register_L(srv: int, L: int, n: int, ldl: int, precision: str = "f32") -> int:
    lid = ctypes.c_int32()
    _check(_lib.trsm_server_register_L(srv, L, n, ldl, PRECISIONS[precision], ctypes.byref(lid)),
           "trsm_server_register_L")
    return lid.value


def trsm_server_register_chol(server: int, L: int, n: int, ldl: int,
                              precision: str = "f32") -> int:
    """Register L as the Cholesky factor of A = L L^T: requests solve A X = B."""
    lid = ctypes.c_int32()
    _check(_lib.trsm_server_register_chol(server, L, n, ldl, PRECISIONS[precision],
                                          ctypes.byref(lid)), "trsm_server_register_chol")
    return lid.value


def trsm_serve_submit(srv: int, l_id: int, B: int, k: int, ldb: int, X: int, ldx: int) -> int:
    t = ctypes.c_uint64()
    _check(_lib.trsm_serve_submit(srv, l_id, B, k, ldb, X, ldx, ctypes.byref(t)),
           "trsm_serve_submit")
    return t.value


def trsm_serve_request_bytes(srv: int, l_id: int, k: int) -> int:
    b = ctypes.c_size_t()
    _check(_lib.trsm_serve_request_bytes(srv, l_id, k, ctypes.byref(b)),
           "trsm_serve_request_bytes")
    return b.value


def trsm_serve_poll(srv: int, ticket: int):
    """(state, status, info): info is the request's Info once it is finished
    (else None); a finished ticket is reported once."""
    st, info = ctypes.c_int(), Info()
    status = _lib.trsm_serve_poll(srv, ticket, ctypes.byref(st), ctypes.byref(info))
    done = st.value in (REQ_DONE, REQ_ERROR)
    return st.value, status, info if done else None


def trsm_server_stats(srv: int) -> ServeStats:
    st = ServeStats()
    _check(_lib.trsm_server_stats(srv, ctypes.byref(st)), "trsm_server_stats")
    return st


def trsm_server_reset_stats(srv: int) -> None:
    _check(_lib.trsm_server_reset_stats(srv), "trsm_server_reset_stats")


def trsm_server_destroy(srv: int) -> None:
    _check(_lib.trsm_server_destroy(srv), "trsm_server_destroy")


def trsm_chol_sizes(n: int, nb: int = 0):
    """(nb_used, linv_bytes, workspace_bytes) of a Cholesky factorization."""
    nbu, lb, wb = ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.trsm_chol_sizes(n, nb, ctypes.byref(nbu), ctypes.byref(lb), ctypes.byref(wb)),
           "trsm_chol_sizes")
    return nbu.value, lb.value, wb.value


def trsm_chol_factor(n: int, A: int, lda: int, nb: int, Linv: int, workspace: int,
                     stream: int = 0) -> None:
    _check(_lib.trsm_chol_factor(n, A, lda, nb, Linv, workspace, stream), "trsm_chol_factor")


def trsm_chol_check(workspace: int):
    """(status, index) of the last factorization on `workspace` (blocking)."""
    st, idx = ctypes.c_int(), ctypes.c_int64()
    _check(_lib.trsm_chol_check(workspace, ctypes.byref(st), ctypes.byref(idx)),
           "trsm_chol_check")
    return st.value, idx.value


def trsm_lu_sizes(n: int, nb: int = 0):
    """(nb_used, inv_bytes per inverse buffer, workspace_bytes) of an LU
    factorization without row exchanges."""
    nbu, lb, wb = ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.trsm_lu_sizes(n, nb, ctypes.byref(nbu), ctypes.byref(lb), ctypes.byref(wb)),
           "trsm_lu_sizes")
    return nbu.value, lb.value, wb.value


def trsm_lu_factor(n: int, A: int, lda: int, nb: int, Linv: int, Uinv: int, workspace: int,
                   stream: int = 0) -> None:
    _check(_lib.trsm_lu_factor(n, A, lda, nb, Linv, Uinv, workspace, stream), "trsm_lu_factor")


def trsm_lu_check(workspace: int):
    """(status, index) of the last LU factorization on `workspace` (blocking)."""
    st, idx = ctypes.c_int(), ctypes.c_int64()
    _check(_lib.trsm_lu_check(workspace, ctypes.byref(st), ctypes.byref(idx)), "trsm_lu_check")
    return st.value, idx.value


def trsm_lu_piv_sizes(n: int, nb: int = 0):
    """(nb_used, Linv bytes, workspace_bytes) of an LU factorization with
    partial pivoting."""
    nbu, lb, wb = ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.trsm_lu_piv_sizes(n, nb, ctypes.byref(nbu), ctypes.byref(lb), ctypes.byref(wb)),
           "trsm_lu_piv_sizes")
    return nbu.value, lb.value, wb.value


def trsm_lu_piv_factor(n: int, A: int, lda: int, nb: int, ipiv: int, Linv: int, workspace: int,
                       stream: int = 0) -> None:
    _check(_lib.trsm_lu_piv_factor(n, A, lda, nb, ipiv, Linv, workspace, stream),
           "trsm_lu_piv_factor")


def trsm_lu_piv_check(workspace: int):
    """(status, index) of the last pivoted LU factorization on `workspace`
    (blocking)."""
    st, idx = ctypes.c_int(), ctypes.c_int64()
    _check(_lib.trsm_lu_piv_check(workspace, ctypes.byref(st), ctypes.byref(idx)),
           "trsm_lu_piv_check")
    return st.value, idx.value


def trsm_row_swaps(k0: int, k1: int, ipiv: int, B: int, ldb: int, ncols: int,
                   stream: int = 0) -> None:
    _check(_lib.trsm_row_swaps(k0, k1, ipiv, B, ldb, ncols, stream), "trsm_row_swaps")


# ---- torch-tensor convenience (memory ownership only) ------------------------

def _stream_handle(torch, device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ld(t) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("matrices must be 2-D with unit column stride (row-major)")
    if t.shape[0] > 1 and t.stride(0) < t.shape[1]:
        raise ValueError("matrix rows overlap (row stride below the column count)")
    return max(t.stride(0), t.shape[1], 1)


def _dev(t, dtype, what: str) -> int:
    """Device pointer of a CUDA tensor of the given dtype; a host tensor or a
    wrong element type is refused before anything reaches the library."""
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{what} must be a CUDA (HIP device) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    return t.data_ptr()


@dataclass
class Solver:
    """Owns a plan plus the Linv and workspace buffers (torch uint8 tensors)."""
    plan: int
    info: PlanInfo
    linv: object
    workspace: object

    @classmethod
    def create(cls, n: int, k: int, precision: str = "f64", n0: int = 0, flags: int = 0,
               device: str = "cuda", tolerance: float = 0.0):
        import torch
        plan = trsm_plan(n, k, PRECISIONS[precision], n0, flags)
        try:
            trsm_plan_set_tolerance(plan, tolerance)
        except Exception:
            trsm_plan_destroy(plan)
            raise
        info = trsm_plan_get_info(plan)
        linv = torch.empty(max(info.linv_bytes, 1) + 256, dtype=torch.uint8, device=device)
        ws = torch.empty(max(info.workspace_bytes, 1) + 256, dtype=torch.uint8, device=device)
        return cls(plan, info, linv, ws)

    @staticmethod
    def _aligned(buf) -> int:
        p = buf.data_ptr()
        return (p + 255) // 256 * 256

    @property
    def linv_ptr(self) -> int:
        return self._aligned(self.linv)

    @property
    def workspace_ptr(self) -> int:
        return self._aligned(self.workspace)

    def _dtype(self):
        import torch
        return torch.float32 if self.info.precision == F32 else torch.float64

    def invert(self, L) -> None:
        import torch
        trsm_invert_diag(self.plan, _dev(L, self._dtype(), "L"), _ld(L), self.linv_ptr,
                         _stream_handle(torch, L.device))

    def solve(self, L, B, X=None, info: Optional[Info] = None, linv_ptr: int = 0) -> object:
        """X = L^{-1} B with this plan's inverted blocks (or, via linv_ptr,
        blocks in the same layout made elsewhere, e.g. by a factorization)."""
        import torch
        if X is None:
            X = torch.empty_like(B)
        dt = self._dtype()
        # TRSM_OK, or TRSM_ENOTCONVERGED (X then holds the last iterate)
        self.last_status = trsm_solve(self.plan, _dev(L, dt, "L"), _ld(L),
                                      linv_ptr or self.linv_ptr, _dev(B, dt, "B"), _ld(B),
                                      _dev(X, dt, "X"), _ld(X), self.workspace_ptr,
                                      _stream_handle(torch, B.device), info)
        return X

    def last_error(self):
        return trsm_plan_last_error(self.plan)

    def close(self):
        if self.plan:
            trsm_plan_destroy(self.plan)
            self.plan = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Cholesky:
    """Owns the Linv and workspace buffers of a Cholesky factorization of one
    size (torch uint8 tensors, 256-byte aligned views)."""

    def __init__(self, n: int, nb: int = 0, device: str = "cuda"):
        import torch
        self.n = n
        self.nb, lb, wb = trsm_chol_sizes(n, nb)
        self._linv = torch.empty(max(lb, 1) + 256, dtype=torch.uint8, device=device)
        self._ws = torch.empty(max(wb, 1) + 256, dtype=torch.uint8, device=device)
        self.linv_bytes = lb

    @property
    def linv_ptr(self) -> int:
        return (self._linv.data_ptr() + 255) // 256 * 256

    @property
    def workspace_ptr(self) -> int:
        return (self._ws.data_ptr() + 255) // 256 * 256

    def factor(self, A) -> None:
        """In place: the lower triangle of the float64 tensor A becomes L."""
        import torch
        if A.shape[0] != self.n or A.shape[1] < self.n:
            raise ValueError("A must be an n x n float64 tensor")
        trsm_chol_factor(self.n, _dev(A, torch.float64, "A"), _ld(A), self.nb, self.linv_ptr,
                         self.workspace_ptr, _stream_handle(torch, A.device))

    def linv_blocks(self):
        """The inverted diagonal blocks as an (m, nb, nb) float64 view."""
        import torch
        m = (self.n + self.nb - 1) // self.nb
        off = self.linv_ptr - self._linv.data_ptr()
        return self._linv[off:off + m * self.nb * self.nb * 8].view(torch.float64).view(
            m, self.nb, self.nb)

    def check(self):
        return trsm_chol_check(self.workspace_ptr)


def cholesky(A, nb: int = 0):
    """L with A = L L^T on the GPU (A float64, symmetric positive definite;
    only its lower triangle is read).  Returns a new tensor, zeros above the
    diagonal; raises TrsmError(ESINGULAR) if A is not positive definite."""
    import torch
    n = A.shape[0]
    L = A.clone()
    c = Cholesky(n, nb, device=A.device)
    c.factor(L)
    st, idx = c.check()
    if st != OK:
        raise TrsmError(st, f"cholesky (row {idx})")
    return L.tril_()


class LU:
    """Owns the Linv, Uinv and workspace buffers of an LU factorization
    without row exchanges of one size (torch uint8 tensors, aligned views)."""

    def __init__(self, n: int, nb: int = 0, device: str = "cuda"):
        import torch
        self.n = n
        self.nb, lb, wb = trsm_lu_sizes(n, nb)
        self._linv = torch.empty(max(lb, 1) + 256, dtype=torch.uint8, device=device)
        self._uinv = torch.empty(max(lb, 1) + 256, dtype=torch.uint8, device=device)
        self._ws = torch.empty(max(wb, 1) + 256, dtype=torch.uint8, device=device)
        self.inv_bytes = lb

    @staticmethod
    def _aligned(buf) -> int:
        return (buf.data_ptr() + 255) // 256 * 256

    @property
    def linv_ptr(self) -> int:
        return self._aligned(self._linv)

    @property
    def uinv_ptr(self) -> int:
        return self._aligned(self._uinv)

    @property
    def workspace_ptr(self) -> int:
        return self._aligned(self._ws)

    def factor(self, A) -> None:
        """In place: A becomes L (strictly lower, unit diagonal implied) and U."""
        import torch
        if A.shape[0] != self.n or A.shape[1] < self.n:
            raise ValueError("A must be an n x n float64 tensor")
        trsm_lu_factor(self.n, _dev(A, torch.float64, "A"), _ld(A), self.nb, self.linv_ptr,
                       self.uinv_ptr, self.workspace_ptr, _stream_handle(torch, A.device))

    def _blocks(self, buf):
        import torch
        m = (self.n + self.nb - 1) // self.nb
        off = self._aligned(buf) - buf.data_ptr()
        return buf[off:off + m * self.nb * self.nb * 8].view(torch.float64).view(
            m, self.nb, self.nb)

    def linv_blocks(self):
        return self._blocks(self._linv)

    def uinv_blocks(self):
        return self._blocks(self._uinv)

    def check(self):
        return trsm_lu_check(self.workspace_ptr)


def lu_nopiv(A, nb: int = 0):
    """(L, U) with A = L U, no row exchanges, on the GPU (A float64).  Raises
    TrsmError(ESINGULAR) at a zero or non-finite pivot."""
    import torch
    n = A.shape[0]
    F = A.clone()
    f = LU(n, nb, device=A.device)
    f.factor(F)
    st, idx = f.check()
    if st != OK:
        raise TrsmError(st, f"lu_nopiv (row {idx})")
    L = torch.tril(F, -1)
    L.diagonal().fill_(1.0)
    return L, torch.triu(F)


class LUPiv:
    """Owns the ipiv, Linv and workspace buffers of an LU factorization with
    partial pivoting of one size (torch tensors, 256-byte aligned views)."""

    def __init__(self, n: int, nb: int = 0, device: str = "cuda"):
        import torch
        self.n = n
        self.nb, lb, wb = trsm_lu_piv_sizes(n, nb)
        self.ipiv = torch.empty(max(n, 1), dtype=torch.int64, device=device)
        self._linv = torch.empty(max(lb, 1) + 256, dtype=torch.uint8, device=device)
        self._ws = torch.empty(max(wb, 1) + 256, dtype=torch.uint8, device=device)

    @staticmethod
    def _aligned(buf) -> int:
        return (buf.data_ptr() + 255) // 256 * 256

    @property
    def linv_ptr(self) -> int:
        return self._aligned(self._linv)

    @property
    def workspace_ptr(self) -> int:
        return self._aligned(self._ws)

    def factor(self, A) -> None:
        """In place: A becomes L (strictly lower, unit diagonal implied) and U
        of P A = L U; self.ipiv the exchanges."""
        import torch
        if A.shape[0] != self.n or A.shape[1] < self.n:
            raise ValueError("A must be an n x n float64 tensor")
        trsm_lu_piv_factor(self.n, _dev(A, torch.float64, "A"), _ld(A), self.nb,
                           self.ipiv.data_ptr(), self.linv_ptr, self.workspace_ptr,
                           _stream_handle(torch, A.device))

    def apply(self, B) -> None:
        """B <- P B, in place (B float64, n rows)."""
        import torch
        trsm_row_swaps(0, self.n, self.ipiv.data_ptr(), _dev(B, torch.float64, "B"), _ld(B),
                       B.shape[1], _stream_handle(torch, B.device))

    def linv_blocks(self):
        import torch
        m = (self.n + self.nb - 1) // self.nb
        off = self.linv_ptr - self._linv.data_ptr()
        return self._linv[off:off + m * self.nb * self.nb * 8].view(torch.float64).view(
            m, self.nb, self.nb)

    def check(self):
        return trsm_lu_piv_check(self.workspace_ptr)


def lu_piv(A, nb: int = 0):
    """(L, U, ipiv) with P A = L U by partial pivoting, on the GPU (A
    float64).  Raises TrsmError(ESINGULAR) at a zero pivot."""
    import torch
    n = A.shape[0]
    F = A.clone()
    f = LUPiv(n, nb, device=A.device)
    f.factor(F)
    st, idx = f.check()
    if st != OK:
        raise TrsmError(st, f"lu_piv (column {idx})")
    L = torch.tril(F, -1)
    L.diagonal().fill_(1.0)
    return L, torch.triu(F), f.ipiv.clone()


def lu_piv_solve(A, B, nb: int = 0):
    """X = A^{-1} B on the GPU (binary64) by LU with partial pivoting: P B,
    then L Y = P B with the factorization's inverted blocks, then U X = Y with
    an upper plan reading U in the factored copy of A."""
    import torch
    n, k = B.shape
    F = A.clone()
    f = LUPiv(n, nb, device=A.device)
    f.factor(F)
    PB = B.clone().contiguous()
    f.apply(PB)
    fwd = Solver.create(n, k, "f64", n0=f.nb, device=B.device)
    up = Solver.create(n, k, "f64", 0, FLAG_UPPER, device=B.device)
    try:
        if fwd.info.n0 != f.nb:
            raise ValueError(f"lu_piv_solve: blocks of {f.nb} rows do not fit a plan for n = {n}")
        Y = fwd.solve(F, PB, linv_ptr=f.linv_ptr)
        up.invert(F)
        X = up.solve(F, Y)
        st, idx = f.check()
        if st != OK:
            raise TrsmError(st, f"lu_piv_solve (column {idx})")
        return X
    finally:
        torch.cuda.current_stream(B.device).synchronize()
        fwd.close()
        up.close()


def lu_solve(A, B, nb: int = 0):
    """X = A^{-1} B on the GPU (binary64) by the LU factorization without row
    exchanges: L Y = B with the factorization's inverted blocks, then U X = Y
    with an upper plan reading U in the factored copy of A.  Raises
    TrsmError(ESINGULAR) at a zero or non-finite pivot."""
    import torch
    n, k = B.shape
    F = A.clone()
    f = LU(n, nb, device=A.device)
    f.factor(F)
    fwd = Solver.create(n, k, "f64", n0=f.nb, device=B.device)
    up = Solver.create(n, k, "f64", 0, FLAG_UPPER, device=B.device)
    if fwd.info.n0 != f.nb:
        # a plan caps n0 at the next power of two >= n (below the 64-row
        # factorization leaf only for n <= 32): the blocks' row stride would
        # not match the plan's
        fwd.close()
        up.close()
        raise ValueError(f"lu_solve: the factorization's {f.nb}-row inverted blocks do not fit "
                         f"a plan for n = {n} (its block size is {fwd.info.n0})")
    try:
        Y = fwd.solve(F, B.contiguous(), linv_ptr=f.linv_ptr)
        up.invert(F)
        X = up.solve(F, Y)
        st, idx = f.check()
        if st != OK:
            raise TrsmError(st, f"lu_solve (row {idx})")
        return X
    finally:
        torch.cuda.current_stream(B.device).synchronize()
        fwd.close()
        up.close()


def solve(L, B, precision: str = "f64", n0: int = 0, flags: int = 0, info: Optional[Info] = None,
          tolerance: float = 0.0):
    """X = L^{-1} B on the GPU: plan, invert the diagonal blocks, sweep
    (mixed precisions: refined to `tolerance`, 0 = binary64's level)."""
    n, k = B.shape
    s = Solver.create(n, k, precision, n0, flags, device=B.device, tolerance=tolerance)
    try:
        if not (flags & FLAG_RECURSIVE):
            s.invert(L)
        return s.solve(L, B, info=info)
    finally:
        import torch
        torch.cuda.current_stream(B.device).synchronize()
        s.close()
