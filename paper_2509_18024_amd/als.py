"""Torch-facing wrapper around the C ABI: holds device tensors and the context.

Only marshalling happens here (shape/dtype/device checks, pointer passing);
all computation runs in libcoreals.so.  The ALS driver alternates the two
half-sweeps in the order of Algorithm 2 (users from M, then items from U).
FoldIn wraps the learned fold-in model (network answers for new users, kept
when the residual of the user's regression is small, exact solves otherwise).
"""
from __future__ import annotations

from typing import Optional, Tuple

import torch

from . import capi


def _need(t: torch.Tensor, dtype, numel: Optional[int], name: str) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


class CoreALS:
    """One problem instance on the current CUDA (HIP) device."""

    def __init__(self, n_u: int, n_m: int, n_f: int, row_ptr: torch.Tensor, col_idx: torch.Tensor,
                 val: torch.Tensor, lam: float, budget: Tuple[int, int] = (1, 1), min_keep: int = 1,
                 precision: int = capi.ALS_PREC_FP32, validate: bool = True, stream=None,
                 heavy_min_degree: int = 0, heavy_chunk: int = 0, heavy_pair_cap: int = 0,
                 light_blocks: int = 0, graphs: bool = False, users_only: bool = False,
                 generic_gathers: bool = False, csc=None, fast: bool = False, unif: bool = False,
                 implicit_alpha: Optional[float] = None):
        capi.load()
        nnz = int(col_idx.numel())
        _need(row_ptr, torch.int64, n_u + 1, "row_ptr")
        _need(col_idx, torch.int32, None, "col_idx")
        _need(val, torch.float32, nnz, "val")
        self.n_u, self.n_m, self.n_f, self.nnz = int(n_u), int(n_m), int(n_f), nnz
        self.device = row_ptr.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._keep = (row_ptr, col_idx, val)
        p = capi.als_problem()
        p.n_u, p.n_m, p.nnz, p.n_f = self.n_u, self.n_m, nnz, self.n_f
        p.row_ptr, p.col_idx, p.val = row_ptr.data_ptr(), col_idx.data_ptr(), val.data_ptr()
        p.lambda_ = float(lam)
        p.budget_num, p.budget_den = int(budget[0]), int(budget[1])
        p.min_keep = int(min_keep)
        p.precision = int(precision)
        p.flags = ((capi.ALS_VALIDATE if validate else 0) | (capi.ALS_USERS_ONLY if users_only else 0)
                   | (capi.ALS_GENERIC_GATHERS if generic_gathers else 0)
                   | (capi.ALS_FAST_VARIANT if fast else 0) | (capi.ALS_UNIF if unif else 0)
                   | (capi.ALS_IMPLICIT if implicit_alpha is not None else 0))
        p.alpha = float(implicit_alpha or 0.0)
        p.stream = self.stream.cuda_stream
        p.heavy_min_degree = int(heavy_min_degree)
        p.heavy_chunk = int(heavy_chunk)
        p.heavy_pair_cap = int(heavy_pair_cap)
        p.light_blocks = int(light_blocks)
        if csc is not None:
            # the caller's column view of the same R (col_ptr, row_idx, val_t)
            cp, ri, vt = csc
            _need(cp, torch.int64, n_m + 1, "col_ptr")
            _need(ri, torch.int32, nnz, "row_idx")
            _need(vt, torch.float32, nnz, "val_t")
            p.col_ptr, p.row_idx, p.val_t = cp.data_ptr(), ri.data_ptr(), vt.data_ptr()
            self._keep = self._keep + (cp, ri, vt)
        size = capi.als_workspace_size(p)
        if size == 0:
            raise capi.ALSError(capi.ALS_E_ARG, "invalid problem sizes")
        self.workspace = torch.empty(size, dtype=torch.uint8, device=self.device)
        p.workspace, p.workspace_bytes = self.workspace.data_ptr(), size
        self.problem = p
        self.ctx = capi.als_init(p)
        if graphs:
            capi.als_use_graphs(self.ctx, True)

    @classmethod
    def from_problem(cls, prob, device="cuda", budget=None, precision=capi.ALS_PREC_FP32, **kw):
        rp = torch.as_tensor(prob.row_ptr, dtype=torch.int64).to(device)
        ci = torch.as_tensor(prob.col_idx, dtype=torch.int32).to(device)
        v = torch.as_tensor(prob.val, dtype=torch.float32).to(device)
        b = budget if budget is not None else (prob.budget_num, prob.budget_den)
        return cls(prob.n_u, prob.n_m, prob.n_f, rp, ci, v, prob.lam, b, prob.min_keep, precision, **kw)

    def half_sweep_users(self, M: torch.Tensor, U: Optional[torch.Tensor] = None, stats: bool = False):
        _need(M, torch.float32, self.n_m * self.n_f, "M")
        if U is None:
            U = torch.empty(self.n_u, self.n_f, dtype=torch.float32, device=self.device)
        _need(U, torch.float32, self.n_u * self.n_f, "U")
        st = capi.half_sweep_users(self.ctx, M.data_ptr(), U.data_ptr(), stats)
        return (U, st) if stats else U

    def half_sweep_items(self, U: torch.Tensor, M: Optional[torch.Tensor] = None, stats: bool = False):
        _need(U, torch.float32, self.n_u * self.n_f, "U")
        if M is None:
            M = torch.empty(self.n_m, self.n_f, dtype=torch.float32, device=self.device)
        _need(M, torch.float32, self.n_m * self.n_f, "M")
        st = capi.half_sweep_items(self.ctx, U.data_ptr(), M.data_ptr(), stats)
        return (M, st) if stats else M

    def core_select(self, side: int, other: torch.Tensor, row_begin: int, row_end: int):
        n_other = self.n_m if side == 0 else self.n_u
        _need(other, torch.float32, n_other * self.n_f, "other")
        cnt = capi.core_select_count(self.ctx, side, row_begin, row_end)
        sel_ptr = torch.empty(row_end - row_begin + 1, dtype=torch.int64, device=self.device)
        sel_pos = torch.empty(max(cnt, 1), dtype=torch.int32, device=self.device)
        capi.core_select(self.ctx, side, other.data_ptr(), row_begin, row_end, sel_ptr.data_ptr(),
                         sel_pos.data_ptr(), cnt)
        return sel_ptr, sel_pos[:cnt]

    def set_sample_seed(self, seed: int) -> None:
        """UNIF: the seed of the following half-sweeps' uniform draws."""
        capi.als_set_sample_seed(self.ctx, seed)

    def core_select_global(self, side: int, other: torch.Tensor):
        """Fast variant: the global cut (T, K) of `other`, int32 [n_f] each."""
        n_other = self.n_m if side == 0 else self.n_u
        _need(other, torch.float32, n_other * self.n_f, "other")
        T = torch.empty(self.n_f, dtype=torch.int32, device=self.device)
        K = torch.empty(self.n_f, dtype=torch.int32, device=self.device)
        capi.core_select_global(self.ctx, side, other.data_ptr(), T.data_ptr(), K.data_ptr())
        return T, K

    def objective(self, U: torch.Tensor, M: torch.Tensor) -> dict:
        _need(U, torch.float32, self.n_u * self.n_f, "U")
        _need(M, torch.float32, self.n_m * self.n_f, "M")
        o = capi.objective(self.ctx, U.data_ptr(), M.data_ptr())
        return {"f": o.f, "sse": o.sse, "rmse": o.rmse, "remse": o.remse}

    def close(self) -> None:
        if getattr(self, "ctx", None):
            capi.als_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_als(als: CoreALS, M0: torch.Tensor, iters: int, record: bool = False):
    """Algorithm 2: for t = 1..iters, U <- users(M), M <- items(U)."""
    M = M0.clone()
    U = torch.empty(als.n_u, als.n_f, dtype=torch.float32, device=als.device)
    hist = []
    for _ in range(iters):
        als.half_sweep_users(M, U)
        if record:
            hist.append(als.objective(U, M))
        als.half_sweep_items(U, M)
        if record:
            hist.append(als.objective(U, M))
    return U, M, hist


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


class FoldIn:
    """Fold-in network 64 -> hidden -> hidden -> 64 (GELU) over the rating-weighted
    embedding bag of item factors, with FP32 master weights in a device workspace."""

    def __init__(self, n_f: int, params: torch.Tensor, hidden: int = 256, max_batch: int = 4096,
                 precision: int = capi.FOLDIN_BF16, max_train_rows: int = 0, lr: float = 1e-3,
                 betas=(0.9, 0.999), eps: float = 1e-8, weight_decay: float = 0.0, stream=None):
        capi.load()
        self.n_f, self.hidden = int(n_f), int(hidden)
        self.P = capi.foldin_param_count(self.n_f, self.hidden)
        _need(params, torch.float32, self.P, "params")
        self.device = params.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        cfg = capi.foldin_cfg()
        cfg.n_f, cfg.hidden, cfg.max_batch, cfg.precision = self.n_f, self.hidden, int(max_batch), int(precision)
        cfg.max_train_rows = int(max_train_rows)
        cfg.lr, cfg.beta1, cfg.beta2, cfg.eps, cfg.weight_decay = lr, betas[0], betas[1], eps, weight_decay
        cfg.stream = self.stream.cuda_stream
        size = capi.foldin_workspace_size(cfg)
        if size == 0:
            raise capi.ALSError(capi.ALS_E_ARG, "invalid fold-in configuration")
        self.workspace = torch.empty(size, dtype=torch.uint8, device=self.device)
        cfg.workspace, cfg.workspace_bytes = self.workspace.data_ptr(), size
        self.cfg = cfg
        self.max_batch = int(max_batch)
        self.m = capi.foldin_create(cfg, params.data_ptr())

    @staticmethod
    def _csr(ptr, items, vals):
        _need(ptr, torch.int64, None, "ptr")
        _need(items, torch.int32, None, "items")
        _need(vals, torch.float32, items.numel(), "vals")
        return ptr.data_ptr(), items.data_ptr(), vals.data_ptr()

    def params(self) -> torch.Tensor:
        out = torch.empty(self.P, dtype=torch.float32, device=self.device)
        capi.foldin_get_params(self.m, out.data_ptr())
        return out

    def set_params(self, params: torch.Tensor) -> None:
        _need(params, torch.float32, self.P, "params")
        capi.foldin_set_params(self.m, params.data_ptr())

    def forward(self, M, ptr, items, vals, rows: Optional[torch.Tensor] = None, n: Optional[int] = None):
        n = int(rows.numel()) if rows is not None else (int(n) if n is not None else ptr.numel() - 1)
        if rows is not None:
            _need(rows, torch.int32, n, "rows")
        _need(M, torch.float32, None, "M")
        out = torch.empty(n, self.n_f, dtype=torch.float32, device=self.device)
        capi.foldin_forward(self.m, M.data_ptr(), *self._csr(ptr, items, vals), _ptr(rows), n, out.data_ptr())
        return out

    def grad(self, M, ptr, items, vals, target, rows: Optional[torch.Tensor] = None, n: Optional[int] = None):
        """Gradient (device [P]) and loss (device [1]) of one batch."""
        n = int(rows.numel()) if rows is not None else int(n)
        if rows is not None:
            _need(rows, torch.int32, n, "rows")
        _need(M, torch.float32, None, "M")
        _need(target, torch.float32, None, "target")
        g = torch.empty(self.P, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        capi.foldin_grad(self.m, M.data_ptr(), *self._csr(ptr, items, vals), _ptr(rows), n, target.data_ptr(),
                         g.data_ptr(), loss.data_ptr())
        return g, loss

    def adamw(self, grad: Optional[torch.Tensor] = None) -> None:
        if grad is not None:
            _need(grad, torch.float32, self.P, "grad")
        capi.foldin_adamw(self.m, _ptr(grad))

    def train(self, M, ptr, items, vals, target, epochs: int, batch: int, seed: int = 0):
        n_rows = ptr.numel() - 1
        _need(M, torch.float32, None, "M")
        _need(target, torch.float32, n_rows * self.n_f, "target")
        return capi.foldin_train(self.m, M.data_ptr(), *self._csr(ptr, items, vals), n_rows, target.data_ptr(),
                                 int(epochs), int(batch), int(seed))

    def answer(self, query: CoreALS, M: torch.Tensor, tol: float = 1e-3, stats: bool = True):
        """(U_new, path, rho, stats) for the users of the query context."""
        _need(M, torch.float32, query.n_m * self.n_f, "M")
        n = query.n_u
        U = torch.empty(n, self.n_f, dtype=torch.float32, device=self.device)
        path = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        rho = torch.empty(max(n, 1), dtype=torch.float32, device=self.device)
        st = capi.foldin_answer(query.ctx, self.m, M.data_ptr(), tol, U.data_ptr(), path.data_ptr(),
                                rho.data_ptr(), stats)
        return U, path[:n], rho[:n], st

    def close(self) -> None:
        if getattr(self, "m", None):
            capi.foldin_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
