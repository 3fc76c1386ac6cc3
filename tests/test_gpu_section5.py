"""The simulation workload of Section 5 at reduced size on the GPU: full ALS,
CORE and UNIF trajectories against the FP64 oracle (same M0, same draws),
and the paper's finding that CORE estimates better than UNIF at the same
rate (Section 5.1), reported as ReMSE and P-ReMSE."""
import numpy as np
import pytest

from paper_2509_18024_amd import synth

gpu = pytest.mark.gpu


@gpu
@pytest.mark.parametrize("dist", ["D1", "D2", "D3"])
def test_section5_core_vs_unif_vs_full(ora, dist):
    import torch
    from paper_2509_18024_amd.als import CoreALS
    prob, held = synth.section5(dist, 400, 400, 20, 0.5, 0.05, seed=620 + int(dist[1]))
    cp, ri, vt = ora.transpose(prob.n_u, prob.n_m, prob.row_ptr, prob.col_idx, prob.val)
    hcp = ora.transpose(prob.n_u, prob.n_m, *held)
    iters = 5
    res = {}
    for method, budget in (("full", (1, 1)), ("core", (1, 10)), ("unif", (1, 10))):
        als = CoreALS.from_problem(prob, "cuda", budget=budget, unif=(method == "unif"))
        M = torch.from_numpy(prob.M0).cuda()
        Mo = prob.M0.astype(np.float64)
        U = torch.empty(prob.n_u, prob.n_f, device="cuda")
        for t in range(iters):
            if method == "unif":
                als.set_sample_seed(2 * t)
                Uo, _ = ora.unif_half_sweep(prob.row_ptr, prob.col_idx, prob.val, Mo, prob.lam, *budget, 1, 2 * t)
            else:
                Uo, _ = ora.half_sweep(prob.row_ptr, prob.col_idx, prob.val, Mo, prob.lam, *budget, 1)
            als.half_sweep_users(M, U)
            if method == "unif":
                als.set_sample_seed(2 * t + 1)
                Mo, _ = ora.unif_half_sweep(cp, ri, vt, Uo, prob.lam, *budget, 1, 2 * t + 1)
            else:
                Mo, _ = ora.half_sweep(cp, ri, vt, Uo, prob.lam, *budget, 1)
            als.half_sweep_items(U, M)
        torch.cuda.synchronize()
        Ug, Mg = U.cpu().numpy().astype(np.float64), M.cpu().numpy().astype(np.float64)
        remse = ora.objective(prob.row_ptr, prob.col_idx, prob.val, Ug, Mg, prob.lam)[3]
        remse_o = ora.objective(prob.row_ptr, prob.col_idx, prob.val, Uo, Mo, prob.lam)[3]
        p_remse = ora.objective(*held, Ug, Mg, prob.lam)[3]
        res[method] = (remse, p_remse)
        print(f"[section5 {dist}] {method}: ReMSE {remse:.5f} (oracle {remse_o:.5f}), P-ReMSE {p_remse:.5f}",
              flush=True)
        # the GPU and the oracle run the same trajectory (same M0, same draws).
        # UNIF's samples hold about n_f entries here (s = 20 for n_f = 20), so
        # its systems are ill-conditioned (D2's factors are all positive and
        # strongly correlated) and the FP32 solves drift further from FP64.
        tol = 5e-2 if method == "unif" else 1e-3
        assert abs(remse - remse_o) <= tol * max(1.0, remse_o)
        als.close()
    # Section 5.1: CORE beats UNIF at the same rate; full ALS is the floor
    assert res["core"][0] < res["unif"][0] and res["core"][1] < res["unif"][1]
    assert res["full"][0] <= res["core"][0]
