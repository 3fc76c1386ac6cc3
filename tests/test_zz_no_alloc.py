"""The allocation-free half-sweep (half_sweep_noalloc) against the workspace
entry points half_sweep_users / half_sweep_items, through the C ABI: two calls
in a row on different problems, the second smaller, each compared with the
workspace entry point on the same inputs (same kernels, same order: the
results must be identical), and the FP32 results also with the FP64 oracle."""
import numpy as np
import pytest

from paper_2509_18024_amd import synth

gpu = pytest.mark.gpu


def rel_fro(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _run_both(als, side, other, n_out, n_f):
    """(workspace result, allocation-free result, stats of each)."""
    import torch
    from paper_2509_18024_amd import capi
    o = torch.from_numpy(np.ascontiguousarray(other)).cuda()
    ref = torch.full((n_out, n_f), 7.0, dtype=torch.float32, device="cuda")
    got = torch.full((n_out, n_f), -7.0, dtype=torch.float32, device="cuda")
    fn = capi.half_sweep_users if side == 0 else capi.half_sweep_items
    st_ref = fn(als.ctx, o.data_ptr(), ref.data_ptr(), True)
    st_got = capi.half_sweep_noalloc(als.ctx, side, o.data_ptr(), got.data_ptr(), True)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy(), st_ref, st_got


def _cases():
    # A: heavy rows split into several chunks and batches (pair cap 64), r = 1/4
    a = synth.random_problem(31, 300, 700, 64, 0.3, budget=(1, 4), heavy_rows=(0, 5, 9, 17))
    # B: smaller, n_f = 48, r = 1/10, one heavy row
    b = synth.random_problem(32, 200, 260, 48, 0.4, budget=(1, 10), heavy_rows=(3,))
    return a, b


@gpu
@pytest.mark.parametrize("precision", [0, 2])
def test_noalloc_matches_workspace_entry_points(ora, precision):
    import torch
    from paper_2509_18024_amd import capi
    from paper_2509_18024_amd.als import CoreALS
    a, b = _cases()
    for k, p in enumerate((a, b)):
        print(f"[noalloc] case {k} n_u={p.n_u} n_m={p.n_m} n_f={p.n_f} precision={precision}", flush=True)
        als = CoreALS.from_problem(p, "cuda", precision=precision, heavy_min_degree=64, heavy_chunk=32,
                                   heavy_pair_cap=64)
        counts = capi.als_class_counts(als.ctx)
        assert counts[0][7] > 0 and counts[1][7] > 0
        U_ref, U_got, s_ref, s_got = _run_both(als, 0, p.M0, p.n_u, p.n_f)
        assert np.array_equal(U_ref, U_got)
        assert (s_ref.n_empty, s_ref.n_singular_fallback, s_ref.n_fp64_residual, s_ref.n_rows) == \
               (s_got.n_empty, s_got.n_singular_fallback, s_got.n_fp64_residual, s_got.n_rows)
        M_ref, M_got, s_ref, s_got = _run_both(als, 1, U_ref, p.n_m, p.n_f)
        assert np.array_equal(M_ref, M_got)
        assert (s_ref.n_singular_fallback, s_ref.n_fp64_residual) == \
               (s_got.n_singular_fallback, s_got.n_fp64_residual)
        Uo, _ = ora.half_sweep(p.row_ptr, p.col_idx, p.val, p.M0.astype(np.float64), p.lam,
                               p.budget_num, p.budget_den, p.min_keep)
        e = rel_fro(U_got, Uo)
        print(f"  users rel err vs oracle {e:.2e}", flush=True)
        assert e <= 1e-4
        als.close()


@gpu
def test_noalloc_rejects_large_pair_cap():
    import torch
    from paper_2509_18024_amd import capi
    from paper_2509_18024_amd.als import CoreALS
    p = synth.random_problem(33, 50, 80, 16, 0.3, budget=(1, 10))
    als = CoreALS.from_problem(p, "cuda")  # default heavy_pair_cap 65536 > 1024
    M = torch.from_numpy(p.M0).cuda()
    U = torch.empty(p.n_u, p.n_f, dtype=torch.float32, device="cuda")
    with pytest.raises(capi.ALSError) as ei:
        capi.half_sweep_noalloc(als.ctx, 0, M.data_ptr(), U.data_ptr())
    assert ei.value.status == capi.ALS_E_ARG
    assert "heavy_pair_cap" in str(ei.value)
    assert capi.half_sweep_noalloc_pair_cap() == 1024
    assert capi.half_sweep_noalloc_scratch_bytes() < 32 << 20
    als.close()
