"""Heavy-row selection that starts from the previous half-sweep's cuts.

The selection (Algorithm 1) of a heavy row may take one counting pass over a
window of 16-bit keys around the same row's threshold of the previous
half-sweep of that side instead of two radix passes; whether the new
threshold lies in the window is decided by exact counts, so the cuts, and
with them the half-sweeps, must not depend on it.  Consecutive half-sweeps of
one context are compared with the FP64 oracle (1e-4 relative Frobenius error,
worst row 1e-3) and with a fresh context (which has no previous cuts): the
two must agree bit for bit."""
import numpy as np
import pytest

from paper_2509_18024_amd import synth

gpu = pytest.mark.gpu

KW = dict(heavy_min_degree=64, heavy_chunk=64, heavy_pair_cap=64)


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


def sequences():
    """(name, problem, factor matrices for consecutive users half-sweeps)."""
    rng = np.random.default_rng(5)
    out = []
    p = synth.random_problem(41, 150, 900, 64, 0.3, budget=(1, 10), heavy_rows=(0, 7))
    M0 = p.M0
    M1 = (M0 * 1.05 + rng.normal(0, 0.02, M0.shape)).astype(np.float32)  # thresholds move a little
    M2 = (M0 * 4.0).astype(np.float32)                                     # they leave the window
    out.append(("nf64_r1/10", p, [M0, M1, M2, M2, M1]))
    p = synth.random_problem(42, 120, 700, 48, 0.3, budget=(1, 4), min_keep=0, heavy_rows=(3,))
    M1 = (p.M0 * 0.9).astype(np.float32)
    out.append(("nf48_r1/4", p, [p.M0, M1, p.M0]))
    # factor entries from a small pool: many keys share the threshold's 16-bit
    # key, so more radix passes and the position pass follow the window
    p = synth.random_problem(43, 100, 800, 64, 0.35, budget=(1, 10), heavy_rows=(1, 2))
    pool = np.array([0.25, -0.5, 0.5, 0.75, -1.0, 1.0, 0.125], np.float32)
    T0 = rng.choice(pool, size=p.M0.shape).astype(np.float32)
    T1 = T0.copy()
    T1[::7] *= np.float32(1.0625)
    out.append(("ties_nf64", p, [T0, T1, T0]))
    return out


@gpu
@pytest.mark.parametrize("which", range(3))
def test_consecutive_half_sweeps_with_previous_cuts(ora, which):
    import torch
    from paper_2509_18024_amd.als import CoreALS
    name, p, Ms = sequences()[which]
    als = CoreALS.from_problem(p, "cuda", **KW)
    hinted = []
    for t, M in enumerate(Ms):
        Mg = torch.from_numpy(M).cuda()
        U, st = als.half_sweep_users(Mg, stats=True)
        fresh = CoreALS.from_problem(p, "cuda", **KW)
        U2, st2 = fresh.half_sweep_users(Mg, stats=True)
        torch.cuda.synchronize()
        fresh.close()
        Uo, so = ora.half_sweep(p.row_ptr, p.col_idx, p.val, M.astype(np.float64), p.lam, p.budget_num,
                                p.budget_den, p.min_keep)
        Ug = U.cpu().numpy()
        hinted.append(st.n_select_hinted)
        note(f"[hint] {name} sweep {t}: hinted rows {st.n_select_hinted} (fresh context {st2.n_select_hinted}), "
             f"rel {rel_fro(Ug, Uo):.2e}, worst row {worst_row(Ug, Uo):.1e}")
        assert st2.n_select_hinted == 0
        assert torch.equal(U, U2)
        assert rel_fro(Ug, Uo) <= 1e-4 and worst_row(Ug, Uo) <= 1e-3
        assert st.n_singular_fallback == so[1]
    assert hinted[0] == 0
    assert max(hinted) > 0  # the window pass ran on some sweep
    als.close()
