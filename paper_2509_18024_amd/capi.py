"""ctypes binding of libcoreals.so (include/coreals.h), same names as the C ABI.

Argument marshalling only: every step runs in the HIP library.  PyTorch is
used for device memory (tensors whose data pointers are passed through) and
for the stream handle.  Importing this module never falls back to anything:
if the library is missing, calls raise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcoreals.so")

ALS_OK, ALS_E_ARG, ALS_E_INDEX, ALS_E_VALUE, ALS_E_NOMEM, ALS_E_DEVICE, ALS_E_STATE = range(7)
ALS_PREC_FP32, ALS_PREC_BF16_IR, ALS_PREC_BF16_IR_FP64RES, ALS_PREC_AUTO = 0, 1, 2, 3
ALS_VALIDATE = 1
ALS_USERS_ONLY = 2
ALS_GENERIC_GATHERS = 4
ALS_FAST_VARIANT = 8
ALS_UNIF = 16
ALS_IMPLICIT = 32
FOLDIN_BF16, FOLDIN_FP32 = 0, 1

STATUS_NAMES = {0: "ALS_OK", 1: "ALS_E_ARG", 2: "ALS_E_INDEX", 3: "ALS_E_VALUE", 4: "ALS_E_NOMEM",
                5: "ALS_E_DEVICE", 6: "ALS_E_STATE"}


class als_problem(ctypes.Structure):
    _fields_ = [
        ("n_u", ctypes.c_int64), ("n_m", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("n_f", ctypes.c_int32),
        ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p),
        ("lambda_", ctypes.c_double),
        ("budget_num", ctypes.c_uint32), ("budget_den", ctypes.c_uint32),
        ("min_keep", ctypes.c_int32), ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
        ("heavy_min_degree", ctypes.c_int32), ("heavy_chunk", ctypes.c_int32),
        ("heavy_pair_cap", ctypes.c_int32), ("light_blocks", ctypes.c_int32),
        ("col_ptr", ctypes.c_void_p), ("row_idx", ctypes.c_void_p), ("val_t", ctypes.c_void_p),
        ("alpha", ctypes.c_double),
    ]


class als_sweep_stats(ctypes.Structure):
    _fields_ = [("n_empty", ctypes.c_int64), ("n_singular_fallback", ctypes.c_int64),
                ("n_fp64_residual", ctypes.c_int64), ("n_rows", ctypes.c_int64),
                ("n_fp32_gram", ctypes.c_int64), ("max_rel_residual", ctypes.c_double),
                ("n_select_hinted", ctypes.c_int64), ("n_pivoted", ctypes.c_int64)]


class als_objective(ctypes.Structure):
    _fields_ = [("f", ctypes.c_double), ("sse", ctypes.c_double), ("rmse", ctypes.c_double),
                ("remse", ctypes.c_double)]


class foldin_cfg(ctypes.Structure):
    _fields_ = [
        ("n_f", ctypes.c_int32), ("hidden", ctypes.c_int32), ("max_batch", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("max_train_rows", ctypes.c_int64),
        ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
        ("eps", ctypes.c_float), ("weight_decay", ctypes.c_float),
        ("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
    ]


class foldin_answer_stats(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_mlp", ctypes.c_int64), ("n_exact", ctypes.c_int64),
                ("n_empty", ctypes.c_int64), ("n_singular_fallback", ctypes.c_int64)]


class ALSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

EXPORTS = ["als_workspace_size", "als_init", "half_sweep_users", "half_sweep_items",
           "core_select_count", "core_select", "objective", "als_profile_begin", "als_profile_end",
           "als_class_counts", "als_use_graphs", "als_destroy", "als_last_error",
           "foldin_param_count", "foldin_workspace_size", "foldin_create", "foldin_get_params",
           "foldin_set_params", "foldin_forward", "foldin_grad", "foldin_adamw", "foldin_train",
           "foldin_answer", "foldin_destroy", "foldin_last_error",
           "half_sweep_noalloc", "half_sweep_noalloc_scratch_bytes", "half_sweep_noalloc_pair_cap",
           "core_select_global", "als_set_sample_seed"]
NCLASS = 8
CLASS_NAMES = ["full", "net1", "net2", "net4", "net8", "net16", "net32", "heavy"]
NPROF = 12
PROF_NAMES = ["full", "net1", "net2", "net4", "net8", "net16", "net32", "heavy_select", "heavy_gram",
              "heavy_solve", "heavy_resid", "heavy_refine"]


def load():
    """Load libcoreals.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build() or python paper_2509_18024_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.als_workspace_size.restype = ctypes.c_size_t
    L.als_workspace_size.argtypes = [ctypes.POINTER(als_problem)]
    L.als_init.restype = i32
    L.als_init.argtypes = [ctypes.POINTER(als_problem), ctypes.POINTER(vp)]
    for name in ("half_sweep_users", "half_sweep_items"):
        f = getattr(L, name)
        f.restype = i32
        f.argtypes = [vp, vp, vp, ctypes.POINTER(als_sweep_stats)]
    L.half_sweep_noalloc.restype = i32
    L.half_sweep_noalloc.argtypes = [vp, i32, vp, vp, ctypes.POINTER(als_sweep_stats)]
    L.half_sweep_noalloc_scratch_bytes.restype = ctypes.c_size_t
    L.half_sweep_noalloc_scratch_bytes.argtypes = []
    L.half_sweep_noalloc_pair_cap.restype = i64
    L.half_sweep_noalloc_pair_cap.argtypes = []
    L.als_set_sample_seed.restype = i32
    L.als_set_sample_seed.argtypes = [vp, ctypes.c_uint64]
    L.core_select_global.restype = i32
    L.core_select_global.argtypes = [vp, i32, vp, vp, vp]
    L.core_select_count.restype = i32
    L.core_select_count.argtypes = [vp, i32, i64, i64, ctypes.POINTER(ctypes.c_int64)]
    L.core_select.restype = i32
    L.core_select.argtypes = [vp, i32, vp, i64, i64, vp, vp, i64]
    L.objective.restype = i32
    L.objective.argtypes = [vp, vp, vp, ctypes.POINTER(als_objective)]
    L.als_profile_begin.restype = i32
    L.als_profile_begin.argtypes = [vp]
    L.als_profile_end.restype = i32
    L.als_profile_end.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.als_class_counts.restype = i32
    L.als_class_counts.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.als_use_graphs.restype = i32
    L.als_use_graphs.argtypes = [vp, i32]
    L.als_destroy.restype = None
    L.als_destroy.argtypes = [vp]
    L.als_last_error.restype = ctypes.c_char_p
    L.als_last_error.argtypes = [vp]
    L.foldin_param_count.restype = i64
    L.foldin_param_count.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.foldin_workspace_size.restype = ctypes.c_size_t
    L.foldin_workspace_size.argtypes = [ctypes.POINTER(foldin_cfg)]
    L.foldin_create.restype = i32
    L.foldin_create.argtypes = [ctypes.POINTER(foldin_cfg), vp, ctypes.POINTER(vp)]
    for name in ("foldin_get_params", "foldin_set_params", "foldin_adamw"):
        f = getattr(L, name)
        f.restype = i32
        f.argtypes = [vp, vp]
    L.foldin_forward.restype = i32
    L.foldin_forward.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp]
    L.foldin_grad.restype = i32
    L.foldin_grad.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp, vp, vp]
    L.foldin_train.restype = i32
    L.foldin_train.argtypes = [vp, vp, vp, vp, vp, i64, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                               ctypes.POINTER(ctypes.c_float)]
    L.foldin_answer.restype = i32
    L.foldin_answer.argtypes = [vp, vp, vp, ctypes.c_double, vp, vp, vp, ctypes.POINTER(foldin_answer_stats)]
    L.foldin_destroy.restype = None
    L.foldin_destroy.argtypes = [vp]
    L.foldin_last_error.restype = ctypes.c_char_p
    L.foldin_last_error.argtypes = [vp]
    _lib = L
    return L


def _check(status: int, ctx) -> None:
    if status != ALS_OK:
        msg = load().als_last_error(ctx)
        raise ALSError(status, msg.decode() if msg else "")


def als_workspace_size(p: als_problem) -> int:
    return int(load().als_workspace_size(ctypes.byref(p)))


def als_init(p: als_problem):
    ctx = ctypes.c_void_p()
    _check(load().als_init(ctypes.byref(p), ctypes.byref(ctx)), None)
    return ctx


def half_sweep_users(ctx, M_ptr: int, U_ptr: int, stats: bool = False):
    st = als_sweep_stats() if stats else None
    _check(load().half_sweep_users(ctx, M_ptr, U_ptr, ctypes.byref(st) if st else None), ctx)
    return st


def half_sweep_items(ctx, U_ptr: int, M_ptr: int, stats: bool = False):
    st = als_sweep_stats() if stats else None
    _check(load().half_sweep_items(ctx, U_ptr, M_ptr, ctypes.byref(st) if st else None), ctx)
    return st


def half_sweep_noalloc(ctx, side: int, other_ptr: int, out_ptr: int, stats: bool = False):
    st = als_sweep_stats() if stats else None
    _check(load().half_sweep_noalloc(ctx, side, other_ptr, out_ptr, ctypes.byref(st) if st else None), ctx)
    return st


def half_sweep_noalloc_scratch_bytes() -> int:
    return int(load().half_sweep_noalloc_scratch_bytes())


def half_sweep_noalloc_pair_cap() -> int:
    return int(load().half_sweep_noalloc_pair_cap())


def core_select_count(ctx, side: int, row_begin: int, row_end: int) -> int:
    out = ctypes.c_int64()
    _check(load().core_select_count(ctx, side, row_begin, row_end, ctypes.byref(out)), ctx)
    return int(out.value)


def core_select(ctx, side: int, other_ptr: int, row_begin: int, row_end: int, sel_ptr_ptr: int,
                sel_pos_ptr: int, sel_cap: int) -> None:
    _check(load().core_select(ctx, side, other_ptr, row_begin, row_end, sel_ptr_ptr, sel_pos_ptr,
                              sel_cap), ctx)


def als_set_sample_seed(ctx, seed: int) -> None:
    _check(load().als_set_sample_seed(ctx, ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF)), ctx)


def core_select_global(ctx, side: int, other_ptr: int, T_ptr: int, K_ptr: int) -> None:
    _check(load().core_select_global(ctx, side, other_ptr, T_ptr, K_ptr), ctx)


def objective(ctx, U_ptr: int, M_ptr: int) -> als_objective:
    out = als_objective()
    _check(load().objective(ctx, U_ptr, M_ptr, ctypes.byref(out)), ctx)
    return out


def als_profile_begin(ctx) -> None:
    _check(load().als_profile_begin(ctx), ctx)


def als_profile_end(ctx):
    """Returns (ms[2][NPROF], launches[2][NPROF]) summed since als_profile_begin."""
    ms = (ctypes.c_double * (2 * NPROF))()
    n = (ctypes.c_int64 * (2 * NPROF))()
    _check(load().als_profile_end(ctx, ms, n), ctx)
    return ([list(ms[:NPROF]), list(ms[NPROF:])], [list(n[:NPROF]), list(n[NPROF:])])


def als_class_counts(ctx):
    out = (ctypes.c_int64 * (2 * NCLASS))()
    _check(load().als_class_counts(ctx, out), ctx)
    return [list(out[:NCLASS]), list(out[NCLASS:])]


def als_use_graphs(ctx, enable: bool) -> None:
    _check(load().als_use_graphs(ctx, 1 if enable else 0), ctx)


def als_destroy(ctx) -> None:
    load().als_destroy(ctx)


def als_last_error(ctx) -> str:
    m = load().als_last_error(ctx)
    return m.decode() if m else ""


# ---------------------------------------------------------------- fold-in

def _fcheck(status: int, model) -> None:
    if status != ALS_OK:
        msg = load().foldin_last_error(model) if model else b"invalid configuration or workspace"
        raise ALSError(status, msg.decode() if msg else "")


def foldin_param_count(n_f: int, hidden: int) -> int:
    return int(load().foldin_param_count(n_f, hidden))


def foldin_workspace_size(cfg: foldin_cfg) -> int:
    return int(load().foldin_workspace_size(ctypes.byref(cfg)))


def foldin_create(cfg: foldin_cfg, params_ptr: int):
    m = ctypes.c_void_p()
    _fcheck(load().foldin_create(ctypes.byref(cfg), params_ptr, ctypes.byref(m)), None)
    return m


def foldin_get_params(m, params_ptr: int) -> None:
    _fcheck(load().foldin_get_params(m, params_ptr), m)


def foldin_set_params(m, params_ptr: int) -> None:
    _fcheck(load().foldin_set_params(m, params_ptr), m)


def foldin_forward(m, M_ptr, ptr_ptr, items_ptr, vals_ptr, rows_ptr, n, out_ptr) -> None:
    _fcheck(load().foldin_forward(m, M_ptr, ptr_ptr, items_ptr, vals_ptr, rows_ptr, n, out_ptr), m)


def foldin_grad(m, M_ptr, ptr_ptr, items_ptr, vals_ptr, rows_ptr, n, target_ptr, grad_ptr, loss_ptr) -> None:
    _fcheck(load().foldin_grad(m, M_ptr, ptr_ptr, items_ptr, vals_ptr, rows_ptr, n, target_ptr, grad_ptr,
                               loss_ptr), m)


def foldin_adamw(m, grad_ptr) -> None:
    _fcheck(load().foldin_adamw(m, grad_ptr), m)


def foldin_train(m, M_ptr, ptr_ptr, items_ptr, vals_ptr, n_rows, target_ptr, epochs, batch, seed):
    losses = (ctypes.c_float * max(epochs, 1))()
    _fcheck(load().foldin_train(m, M_ptr, ptr_ptr, items_ptr, vals_ptr, n_rows, target_ptr, epochs, batch,
                                seed, losses), m)
    return list(losses[:epochs])


def foldin_answer(ctx, m, M_ptr, tol, U_ptr, path_ptr, rho_ptr, stats: bool = False):
    st = foldin_answer_stats() if stats else None
    _fcheck(load().foldin_answer(ctx, m, M_ptr, float(tol), U_ptr, path_ptr, rho_ptr,
                                 ctypes.byref(st) if st else None), m)
    return st


def foldin_destroy(m) -> None:
    load().foldin_destroy(m)
