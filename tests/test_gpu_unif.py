"""UNIF, the uniform-subsampling comparator of Section 5, against the FP64
oracle: the same draws (splitmix64 keys on both sides, written separately
from the generator's published definition) and the sample's ridge system,
within 1e-4 relative Frobenius error per half-sweep."""
import numpy as np
import pytest

from paper_2509_18024_amd import synth

gpu = pytest.mark.gpu


def rel_fro(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def unif_cases():
    return [
        ("nf64_r1/10", synth.random_problem(91, 300, 500, 64, 0.1, budget=(1, 10), heavy_rows=(2, 9)),
         dict(heavy_min_degree=64, heavy_chunk=64, heavy_pair_cap=16), 3),
        ("nf32_r1/4", synth.random_problem(92, 200, 260, 32, 0.2, budget=(1, 4)), {}, 12345),
        ("nf48_r1/10_minkeep0", synth.random_problem(93, 250, 300, 48, 0.15, budget=(1, 10), min_keep=0,
                                                     heavy_rows=(0,)), dict(heavy_min_degree=64), 7),
    ]


@gpu
@pytest.mark.parametrize("which", range(3))
def test_unif_half_sweeps_match_oracle(ora, which):
    import torch
    from paper_2509_18024_amd.als import CoreALS
    name, p, kw, seed = unif_cases()[which]
    als = CoreALS.from_problem(p, "cuda", unif=True, **kw)
    als.set_sample_seed(seed)
    U, st = als.half_sweep_users(torch.from_numpy(p.M0).cuda(), stats=True)
    torch.cuda.synchronize()
    Uo, so = ora.unif_half_sweep(p.row_ptr, p.col_idx, p.val, p.M0.astype(np.float64), p.lam, p.budget_num,
                                 p.budget_den, p.min_keep, seed)
    U32 = Uo.astype(np.float32)
    M, st2 = als.half_sweep_items(torch.from_numpy(U32).cuda(), stats=True)
    torch.cuda.synchronize()
    cp, ri, vt = ora.transpose(p.n_u, p.n_m, p.row_ptr, p.col_idx, p.val)
    Mo, smo = ora.unif_half_sweep(cp, ri, vt, U32.astype(np.float64), p.lam, p.budget_num, p.budget_den,
                                  p.min_keep, seed)
    eu, em = rel_fro(U.cpu().numpy(), Uo), rel_fro(M.cpu().numpy(), Mo)
    print(f"[unif] {name} seed {seed}: users {eu:.2e}, items {em:.2e}; singular {st.n_singular_fallback}/{so[1]}, "
          f"{st2.n_singular_fallback}/{smo[1]}", flush=True)
    assert eu <= 1e-4 and em <= 1e-4
    assert st.n_empty == so[0] and st2.n_empty == smo[0]
    assert st.n_singular_fallback == so[1] and st2.n_singular_fallback == smo[1]
    # another seed draws other samples: the factors change
    als.set_sample_seed(seed + 1)
    U2 = als.half_sweep_users(torch.from_numpy(p.M0).cuda())
    torch.cuda.synchronize()
    assert rel_fro(U2.cpu().numpy(), Uo) > 1e-3
    als.close()


@gpu
def test_unif_graph_replay_follows_the_seed(ora):
    """Captured half-sweeps are recaptured when the seed changes."""
    import torch
    from paper_2509_18024_amd.als import CoreALS
    p = synth.random_problem(94, 200, 300, 32, 0.15, budget=(1, 4))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        als = CoreALS.from_problem(p, "cuda", unif=True, stream=stream, graphs=True)
        M = torch.from_numpy(p.M0).cuda()
        outs = []
        for seed in (5, 6, 5):
            als.set_sample_seed(seed)
            U = als.half_sweep_users(M, torch.empty(p.n_u, p.n_f, device="cuda"))
            stream.synchronize()
            outs.append(U.cpu().numpy())
    for seed, U in zip((5, 6, 5), outs):
        Uo, _ = ora.unif_half_sweep(p.row_ptr, p.col_idx, p.val, p.M0.astype(np.float64), p.lam, 1, 4, 1, seed)
        assert rel_fro(U, Uo) <= 1e-4
    als.close()
