"""Implicit-feedback Core-ALS (Section 3, last paragraph) against the FP64
oracle: the ratings are confidences, a row solves
(Y^T Y + X*^T W X + lambda E) u = X*^T (1 + alpha r) with W = diag(alpha r)
and X* the row's core elements (Algorithm 1).  The FP32 bound of the
explicit method applies (1e-4 relative Frobenius error, worst row 1e-3), and
the counts of empty rows and singular core systems agree exactly."""
import dataclasses

import numpy as np
import pytest

from paper_2509_18024_amd import synth

gpu = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)


def rel_fro(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def worst_row(G, O):
    num = np.linalg.norm(np.asarray(G, np.float64) - O, axis=1)
    den = np.linalg.norm(O, axis=1)
    rel = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num > 0, np.inf, 0.0))
    return float(rel.max())


def counts(p, seed):
    """The same mask with interaction counts (1 .. 5) for ratings."""
    rng = np.random.default_rng(seed)
    return dataclasses.replace(p, val=rng.integers(1, 6, size=len(p.val)).astype(np.float32))


def implicit_cases():
    out = []
    p = counts(synth.random_problem(101, 300, 500, 64, 0.08, budget=(1, 10), heavy_rows=(3, 7)), 1)
    # rows 3 and 7 hold all 500 items: heavy rows (degree >= 64), 8 chunks each
    out.append(("nf64_r1/10_heavy", p, 2.0, dict(heavy_min_degree=64, heavy_chunk=64, heavy_pair_cap=16)))
    p = counts(synth.random_problem(102, 200, 260, 32, 0.2, budget=(1, 1), heavy_rows=(0,)), 2)
    out.append(("nf32_r1_implicit_als", p, 40.0, dict(heavy_min_degree=128)))
    p = counts(synth.random_problem(103, 250, 300, 48, 0.15, budget=(1, 4), min_keep=0, heavy_rows=(5,)), 3)
    out.append(("nf48_r1/4_minkeep0", p, 1.0, dict(heavy_min_degree=64)))
    p = counts(synth.random_problem(104, 400, 300, 16, 0.05, budget=(1, 2)), 4)
    out.append(("nf16_r1/2_light", p, 10.0, {}))
    return out


@gpu
@pytest.mark.parametrize("which", range(4))
def test_implicit_half_sweeps_match_oracle(ora, which):
    import torch
    from paper_2509_18024_amd.als import CoreALS
    name, p, alpha, kw = implicit_cases()[which]
    als = CoreALS.from_problem(p, "cuda", implicit_alpha=alpha, **kw)
    U, st = als.half_sweep_users(torch.from_numpy(p.M0).cuda(), stats=True)
    torch.cuda.synchronize()
    Uo, so = ora.implicit_half_sweep(p.row_ptr, p.col_idx, p.val, p.M0.astype(np.float64), p.lam, alpha,
                                     p.budget_num, p.budget_den, p.min_keep)
    U32 = Uo.astype(np.float32)
    M, st2 = als.half_sweep_items(torch.from_numpy(U32).cuda(), stats=True)
    torch.cuda.synchronize()
    cp, ri, vt = ora.transpose(p.n_u, p.n_m, p.row_ptr, p.col_idx, p.val)
    Mo, smo = ora.implicit_half_sweep(cp, ri, vt, U32.astype(np.float64), p.lam, alpha, p.budget_num,
                                      p.budget_den, p.min_keep)
    Ug, Mg = U.cpu().numpy(), M.cpu().numpy()
    note(f"[implicit] {name} alpha={alpha}: users {rel_fro(Ug, Uo):.2e} (worst row {worst_row(Ug, Uo):.1e}), "
         f"items {rel_fro(Mg, Mo):.2e} (worst row {worst_row(Mg, Mo):.1e}); "
         f"fallback {st.n_singular_fallback}/{so[1]}, {st2.n_singular_fallback}/{smo[1]}")
    assert rel_fro(Ug, Uo) <= 1e-4 and rel_fro(Mg, Mo) <= 1e-4
    assert worst_row(Ug, Uo) <= 1e-3 and worst_row(Mg, Mo) <= 1e-3
    assert st.n_empty == so[0] and st.n_singular_fallback == so[1]
    assert st2.n_empty == smo[0] and st2.n_singular_fallback == smo[1]
    als.close()


@gpu
def test_implicit_alpha_zero_is_ridge_on_the_full_gram():
    """alpha = 0: the observed entries carry no weight, so every row's matrix
    is Y^T Y + lambda E and the right-hand side of column a sums the row's s
    kept factor entries of column a: those of largest |x| (ties: the earlier
    entry), s = budget(n).  Computed here with a sort, not with the oracle."""
    import torch
    from paper_2509_18024_amd.als import CoreALS
    p = counts(synth.random_problem(105, 120, 200, 24, 0.1, budget=(1, 10)), 5)
    als = CoreALS.from_problem(p, "cuda", implicit_alpha=0.0)
    U = als.half_sweep_users(torch.from_numpy(p.M0).cuda()).cpu().numpy()
    Y = p.M0.astype(np.float64)
    A = Y.T @ Y + p.lam * np.eye(p.n_f)
    B = np.zeros((p.n_u, p.n_f))
    for i in range(p.n_u):
        Yi = Y[p.col_idx[p.row_ptr[i]:p.row_ptr[i + 1]]]
        n = Yi.shape[0]
        s = max(min(n, p.min_keep), n * p.budget_num // p.budget_den)
        for a in range(p.n_f):
            order = np.argsort(-np.abs(Yi[:, a]), kind="stable")
            B[i, a] = Yi[order[:s], a].sum()
    ref = np.linalg.solve(A, B.T).T
    e = rel_fro(U, ref)
    note(f"[implicit alpha=0] {e:.2e}")
    assert e <= 1e-4
    als.close()


@gpu
def test_implicit_rejections():
    import torch
    from paper_2509_18024_amd import capi
    from paper_2509_18024_amd.als import CoreALS
    p = counts(synth.random_problem(106, 40, 50, 16, 0.3, budget=(1, 4)), 6)
    for kw in (dict(precision=capi.ALS_PREC_BF16_IR), dict(fast=True), dict(unif=True)):
        with pytest.raises(capi.ALSError) as ei:
            CoreALS.from_problem(p, "cuda", implicit_alpha=1.0, **kw)
        assert ei.value.status == capi.ALS_E_ARG
    with pytest.raises(capi.ALSError) as ei:
        CoreALS.from_problem(p, "cuda", implicit_alpha=-1.0)
    assert ei.value.status == capi.ALS_E_ARG
    als = CoreALS.from_problem(p, "cuda", implicit_alpha=1.0)
    M = torch.from_numpy(p.M0).cuda()
    U = torch.empty(p.n_u, p.n_f, device="cuda")
    with pytest.raises(capi.ALSError) as ei:
        capi.half_sweep_noalloc(als.ctx, 0, M.data_ptr(), U.data_ptr())
    assert ei.value.status == capi.ALS_E_ARG
    with pytest.raises(capi.ALSError) as ei:
        als.objective(U, M)
    assert ei.value.status == capi.ALS_E_STATE
    als.close()
