"""Precision modes at rank 128 on the precision-sweep recipe (reduced scale).

The recipe: uniform entries, no noise, ground-truth factors whose singular
values are log-spaced from 1 to 1e3, lambda in {1e-4, 1e-2}, r in {1, 1/10}.
Each configuration runs one users half-sweep from the ground-truth item
factors (the scale the factors reach as ALS converges, where the row systems
are worst conditioned) and one items half-sweep from the oracle's users,
in FP32, BF16 + refinement with an FP32 residual, with an FP64 residual, and
the per-row mode (ALS_PREC_AUTO), and prints the error of each factor matrix
against the FP64 oracle.

The paper fixes no precision, so these errors are not pinned to a value of
the paper.  What the tests hold, from the arithmetic:
  - well-conditioned rows (lambda = 1e-2, r = 1: kappa about 1e2): every
    mode within 1e-4;
  - the per-row mode is never worse than about the FP32 path: rows whose
    condition estimate exceeds 2^8 (where one refinement step from a bf16
    Gram cannot contract) get an FP32-product Gram, so its error is within
    twice the FP32 error (or 1e-4);
  - the FP64 residual is chosen only at lambda < 1e-3.
"""
import dataclasses

import numpy as np
import pytest

from paper_2509_18024_amd import synth

gpu = pytest.mark.gpu
MODES = {0: "fp32", 1: "bf16+IR fp32res", 2: "bf16+IR fp64res", 3: "auto"}


def rel_fro(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def c4():
    return synth.c4_precision(scale=0.01)


@gpu
@pytest.mark.parametrize("lam", [1e-4, 1e-2])
@pytest.mark.parametrize("budget", [(1, 1), (1, 10)])
def test_c4_precision_modes(ora, c4, lam, budget):
    import torch
    from paper_2509_18024_amd.als import CoreALS
    p = dataclasses.replace(c4, lam=lam)
    Mt = p.V_true.astype(np.float32)
    Uo, so = ora.half_sweep(p.row_ptr, p.col_idx, p.val, Mt.astype(np.float64), lam, budget[0], budget[1], 1)
    U32 = Uo.astype(np.float32)
    cp, ri, vt = ora.transpose(p.n_u, p.n_m, p.row_ptr, p.col_idx, p.val)
    Mo, smo = ora.half_sweep(cp, ri, vt, U32.astype(np.float64), lam, budget[0], budget[1], 1)
    errs = {}
    for prec in MODES:
        als = CoreALS.from_problem(p, "cuda", budget=budget, precision=prec)
        U, st = als.half_sweep_users(torch.from_numpy(Mt).cuda(), stats=True)
        M, st2 = als.half_sweep_items(torch.from_numpy(U32).cuda(), stats=True)
        torch.cuda.synchronize()
        eu, em = rel_fro(U.cpu().numpy(), Uo), rel_fro(M.cpu().numpy(), Mo)
        errs[prec] = (eu, em)
        print(f"[c4 n_f=128 lambda={lam:g} r={budget[0]}/{budget[1]}] {MODES[prec]:>16}: U err {eu:.2e}, "
              f"M err {em:.2e}; fp64-residual rows {st.n_fp64_residual}/{st2.n_fp64_residual}, "
              f"fp32-Gram rows {st.n_fp32_gram}/{st2.n_fp32_gram}, singular {st.n_singular_fallback}/"
              f"{st2.n_singular_fallback} (oracle {so[1]}/{smo[1]})", flush=True)
        if prec == 3 and lam >= 1e-3:
            assert st.n_fp64_residual == 0 and st2.n_fp64_residual == 0
        if prec == 2:
            assert st.n_fp64_residual > 0 and st2.n_fp64_residual > 0
        if prec in (0, 1):
            assert st.n_fp64_residual == 0 and st.n_fp32_gram == 0
        als.close()
    if lam == 1e-2 and budget == (1, 1):
        for prec, (eu, em) in errs.items():
            assert eu <= 1e-4 and em <= 1e-4, (MODES[prec], eu, em)
    for k in (0, 1):  # U, M
        assert errs[3][k] <= max(2.0 * errs[0][k], 1e-4), ("auto", k, errs[3][k], errs[0][k])
