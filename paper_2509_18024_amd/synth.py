"""Seeded synthetic inputs for core-elements ALS.

This module only draws inputs: rating matrices in CSR form, ground-truth
factors and the initial item factors M0.  It holds none of the method's
arithmetic (no selection, no Gram, no solve), so both the HIP path and the
FP64 oracle can consume what it produces without sharing any computation.

Every generator takes an explicit seed and uses NumPy's PCG64 stream, so a
(config, scale, seed) triple always yields bit-identical arrays.

Workloads follow the problem statement of the paper (Section 2.1): a rating
matrix R with a set I of observed entries, rank n_f, weighted penalty lambda
and a subsampling rate r.  The public datasets of the paper (Netflix, bark
textures) are not available; the configurations below stand in for them with
synthetic matrices of the same kind (low rank plus noise, heavy-tailed user
and item degrees).

Column sampling without replacement uses systematic probability-proportional-
to-size sampling: for a row of degree d the inclusion probability of column j
is pi_j = min(1, c * p_j) with c chosen so that sum_j pi_j = d; one uniform
offset U then selects the columns whose cumulative pi interval contains one of
U, U+1, ..., U+d-1.  Since every pi_j <= 1 this gives exactly d distinct
columns, already in ascending order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Problem:
    """One ALS problem instance (all arrays on the host)."""

    name: str
    n_u: int
    n_m: int
    n_f: int
    row_ptr: np.ndarray  # int64 [n_u + 1]
    col_idx: np.ndarray  # int32 [nnz], strictly increasing within a row
    val: np.ndarray      # float32 [nnz]
    lam: float
    budget_num: int
    budget_den: int
    min_keep: int
    iters: int
    M0: np.ndarray       # float32 [n_m, n_f], initial item factors
    U_true: Optional[np.ndarray] = None
    V_true: Optional[np.ndarray] = None
    item_p: Optional[np.ndarray] = None  # item popularity used to draw the columns

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def with_budget(self, num: int, den: int, min_keep: Optional[int] = None) -> "Problem":
        q = dataclasses.replace(self, budget_num=int(num), budget_den=int(den))
        if min_keep is not None:
            q.min_keep = int(min_keep)
        return q


# ----------------------------------------------------------------------------
# degree and popularity distributions
# ----------------------------------------------------------------------------

def zipf_weights(rng: np.random.Generator, n: int, s: float) -> np.ndarray:
    """Popularity weights rank^-s, assigned to a random permutation of ids."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    return w[rng.permutation(n)]


def waterfill(p: np.ndarray, cap: float) -> np.ndarray:
    """Clip probabilities at `cap` and give the excess to the unclipped ones."""
    p = p / p.sum()
    if cap * len(p) < 1.0:
        raise ValueError("cap too small for a probability vector")
    for _ in range(200):
        over = p > cap
        if not over.any():
            break
        excess = (p[over] - cap).sum()
        p[over] = cap
        free = p < cap
        p[free] += excess * p[free] / p[free].sum()
    return p / p.sum()


def lomax_degrees(rng, n, alpha, scale, dmax):
    """d = min(dmax, 1 + floor(Lomax(alpha, scale)))."""
    x = rng.pareto(alpha, size=n) * scale
    return np.minimum(dmax, 1 + np.floor(x)).astype(np.int64)


def lognormal_degrees(rng, n, mu, sigma, dmin, dmax):
    x = np.round(rng.lognormal(mu, sigma, size=n))
    return np.clip(x, dmin, dmax).astype(np.int64)


# ----------------------------------------------------------------------------
# sampling distinct columns per row (systematic PPS sampling)
# ----------------------------------------------------------------------------

def _capped_scale(p_sorted_desc: np.ndarray, prefix: np.ndarray, d: np.ndarray) -> np.ndarray:
    """For each degree d find c with sum_j min(1, c p_j) = d (vectorised).

    m = number of capped columns; c_m = (d - m) / (1 - prefix[m]) must satisfy
    c_m * p[m] <= 1 (largest uncapped stays below 1).  The smallest such m wins.
    """
    n = len(p_sorted_desc)
    lo = np.zeros(len(d), dtype=np.int64)
    hi = np.minimum(d, n - 1).astype(np.int64)
    tail = lambda m: np.maximum(1.0 - prefix[m], 1e-300)
    for _ in range(64):
        if np.all(lo >= hi):
            break
        mid = (lo + hi) // 2
        c = (d - mid) / tail(mid)
        ok = c * p_sorted_desc[mid] <= 1.0 + 1e-12
        hi = np.where(ok, mid, hi)
        lo = np.where(ok, lo, mid + 1)
    return (d - lo) / tail(lo)


def sample_rows_pps(rng: np.random.Generator, degrees: np.ndarray, p: np.ndarray,
                    chunk_entries: int = 1 << 24):
    """CSR (row_ptr, col_idx) with row i holding degrees[i] distinct columns."""
    n_rows = len(degrees)
    n_cols = len(p)
    degrees = np.minimum(degrees, n_cols).astype(np.int64)
    p = p / p.sum()
    pmax = p.max()
    light = degrees * pmax <= 1.0
    offsets = rng.random(n_rows)
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(degrees, out=row_ptr[1:])
    col_idx = np.empty(int(row_ptr[-1]), dtype=np.int32)

    # light rows: pi_j = d p_j <= 1, one shared cumulative distribution
    cdf = np.cumsum(p)
    cdf[-1] = max(cdf[-1], 1.0)
    idx = np.nonzero(light)[0]
    start = 0
    while start < len(idx):
        # group consecutive light rows into about chunk_entries entries
        stop = start
        acc = 0
        while stop < len(idx) and (acc < chunk_entries or stop == start):
            acc += degrees[idx[stop]]
            stop += 1
        rows = idx[start:stop]
        d = degrees[rows]
        tot = int(d.sum())
        if tot:
            rep = np.repeat(np.arange(len(rows)), d)
            first = np.zeros(len(rows), dtype=np.int64)
            np.cumsum(d[:-1], out=first[1:])
            k = np.arange(tot, dtype=np.int64) - first[rep]
            q = (offsets[rows][rep] + k) / d[rep]
            cols = np.searchsorted(cdf, q, side="right")
            np.minimum(cols, n_cols - 1, out=cols)
            col_idx[_dest_index(row_ptr, rows, d)] = cols.astype(np.int32)
        start = stop

    # heavy rows: per-row capped inclusion probabilities
    hidx = np.nonzero(~light)[0]
    if len(hidx):
        order = np.argsort(-p, kind="stable")
        ps = p[order]
        prefix = np.concatenate([[0.0], np.cumsum(ps)])
        c_all = _capped_scale(ps, prefix, degrees[hidx].astype(np.float64))
        per = max(1, int(chunk_entries // n_cols))
        for s0 in range(0, len(hidx), per):
            rows = hidx[s0:s0 + per]
            c = c_all[s0:s0 + per]
            pi = np.minimum(1.0, c[:, None] * p[None, :])
            cum = np.cumsum(pi, axis=1)
            big = float(n_cols + 2)
            flat = (cum + big * np.arange(len(rows))[:, None]).ravel()
            d = degrees[rows]
            rep = np.repeat(np.arange(len(rows)), d)
            first = np.zeros(len(rows), dtype=np.int64)
            np.cumsum(d[:-1], out=first[1:])
            k = np.arange(int(d.sum()), dtype=np.int64) - first[rep]
            q = offsets[rows][rep] + k + big * rep
            pos = np.searchsorted(flat, q, side="right")
            cols = pos - rep * n_cols
            np.clip(cols, 0, n_cols - 1, out=cols)
            col_idx[_dest_index(row_ptr, rows, d)] = cols.astype(np.int32)

    return _dedupe(row_ptr, col_idx)


def _dest_index(row_ptr, rows, d):
    rep = np.repeat(np.arange(len(rows)), d)
    first = np.zeros(len(rows), dtype=np.int64)
    np.cumsum(d[:-1], out=first[1:])
    k = np.arange(int(d.sum()), dtype=np.int64) - first[rep]
    return row_ptr[rows][rep] + k


def _dedupe(row_ptr, col_idx):
    """Drop the (floating-point edge case) repeated columns inside a row."""
    n_rows = len(row_ptr) - 1
    nnz = len(col_idx)
    if nnz == 0:
        return row_ptr, col_idx
    row_of = np.repeat(np.arange(n_rows), np.diff(row_ptr))
    keep = np.ones(nnz, dtype=bool)
    same_row = row_of[1:] == row_of[:-1]
    keep[1:] = ~(same_row & (col_idx[1:] <= col_idx[:-1]))
    if keep.all():
        return row_ptr, col_idx
    counts = np.bincount(row_of[keep], minlength=n_rows)
    rp = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return rp, np.ascontiguousarray(col_idx[keep])


def rows_of(row_ptr: np.ndarray) -> np.ndarray:
    return np.repeat(np.arange(len(row_ptr) - 1, dtype=np.int64), np.diff(row_ptr))


def low_rank_values(U: np.ndarray, V: np.ndarray, row_ptr: np.ndarray, col_idx: np.ndarray,
                    chunk: int = 1 << 21) -> np.ndarray:
    """r_ij = U[i] . V[j] on the observed entries (float64 accumulation)."""
    nnz = len(col_idx)
    out = np.empty(nnz, dtype=np.float64)
    r = rows_of(row_ptr)
    try:
        import torch
        Ut = torch.from_numpy(np.ascontiguousarray(U, dtype=np.float64))
        Vt = torch.from_numpy(np.ascontiguousarray(V, dtype=np.float64))
        for s in range(0, nnz, chunk):
            ri = torch.from_numpy(r[s:s + chunk])
            ci = torch.from_numpy(col_idx[s:s + chunk].astype(np.int64))
            out[s:s + chunk] = (Ut[ri] * Vt[ci]).sum(1).numpy()
    except ImportError:  # pragma: no cover - numpy fallback for input synthesis
        for s in range(0, nnz, chunk):
            out[s:s + chunk] = np.einsum("ij,ij->i", U[r[s:s + chunk]], V[col_idx[s:s + chunk]])
    return out


def init_factors(seed: int, n: int, n_f: int, sd: float = 0.1) -> np.ndarray:
    """Initial factor matrix, entries N(0, sd^2), float32."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, sd, size=(n, n_f)).astype(np.float32)


def mean3_factors(rng, n, n_f):
    """Column 0 = sqrt(3), other entries N(0, (n_f-1)^-1/2): U.V has mean 3, sd ~1."""
    F = np.empty((n, n_f), dtype=np.float64)
    F[:, 0] = math.sqrt(3.0)
    if n_f > 1:
        F[:, 1:] = rng.normal(0.0, (n_f - 1) ** -0.25, size=(n, n_f - 1))
    return F


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------

def c1_plain(seed: int = 101, m0_seed: int = 102) -> Problem:
    """Plain full-data ALS: 1000 x 500, n_f = 10, Bernoulli(0.05) mask,
    U0, V0 ~ N(0, 1/n_f), noise N(0, 0.1^2), lambda = 0.05, r = 1, 10 iterations."""
    n_u, n_m, n_f = 1000, 500, 10
    rng = np.random.default_rng(seed)
    U0 = rng.normal(0.0, 1.0 / math.sqrt(n_f), size=(n_u, n_f))
    V0 = rng.normal(0.0, 1.0 / math.sqrt(n_f), size=(n_m, n_f))
    mask = rng.random((n_u, n_m)) < 0.05
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(n_u + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n_u), out=row_ptr[1:])
    col_idx = cols.astype(np.int32)
    val = low_rank_values(U0, V0, row_ptr, col_idx) + rng.normal(0.0, 0.1, size=len(col_idx))
    return Problem("c1_plain", n_u, n_m, n_f, row_ptr, col_idx, val.astype(np.float32),
                   0.05, 1, 1, 1, 10, init_factors(m0_seed, n_m, n_f), U0, V0)


def c2_core(scale: float = 1.0, seed: int = 201, m0_seed: int = 202) -> Problem:
    """Core-elements ALS: 100k x 20k, n_f = 32, user degree LogNormal(4,1) clipped
    to [1, 20000], item popularity Zipf(1.2), ratings round(clip(UV' + N(0,0.25),1,5)),
    r = 1/10, lambda = 0.05, 15 iterations."""
    n_u = max(8, int(round(100_000 * scale)))
    n_m = max(8, int(round(20_000 * scale)))
    n_f = 32
    rng = np.random.default_rng(seed)
    deg = lognormal_degrees(rng, n_u, 4.0, 1.0, 1, min(20_000, n_m))
    p = zipf_weights(rng, n_m, 1.2)
    p = waterfill(p / p.sum(), min(1.0, n_u / max(1, deg.sum())))
    row_ptr, col_idx = sample_rows_pps(rng, deg, p)
    U0 = mean3_factors(rng, n_u, n_f)
    V0 = mean3_factors(rng, n_m, n_f)
    raw = low_rank_values(U0, V0, row_ptr, col_idx) + rng.normal(0.0, 0.5, size=len(col_idx))
    val = np.round(np.clip(raw, 1.0, 5.0)).astype(np.float32)
    return Problem("c2_core", n_u, n_m, n_f, row_ptr, col_idx, val, 0.05, 1, 10, 1, 15,
                   init_factors(m0_seed, n_m, n_f), U0, V0)


def c3_scale_lomax(n_u: int, target_nnz: float, alpha: float = 1.5, dmax: int = 50_000) -> float:
    """Lomax scale giving E[min(dmax, 1 + floor(X))] * n_u ~= target (numeric)."""
    rng = np.random.default_rng(12345)
    z = rng.pareto(alpha, size=400_000)
    lo, hi = 1.0, 1000.0
    goal = target_nnz / n_u
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        m = np.minimum(dmax, 1 + np.floor(z * mid)).mean()
        if m < goal:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def c3_batched(scale: float = 1.0, seed: int = 301, m0_seed: int = 302,
               budget=(1, 10)) -> Problem:
    """Batched uneven solves: 1M x 100k, n_f = 64, ~1e8 entries, user degree
    1 + floor(Lomax(1.5)) capped at 50k, item popularity Zipf(1.1) water-filled so
    that no expected item degree exceeds 50k, fp32 values UV' + N(0, 0.25)."""
    n_u = max(16, int(round(1_000_000 * scale)))
    n_m = max(16, int(round(100_000 * scale)))
    n_f = 64
    target = 1.0e8 * scale
    dmax = min(50_000, n_m)
    lscale = c3_scale_lomax(n_u, target, 1.5, dmax)
    rng = np.random.default_rng(seed)
    deg = lomax_degrees(rng, n_u, 1.5, lscale, dmax)
    p = zipf_weights(rng, n_m, 1.1)
    p = waterfill(p / p.sum(), min(1.0, 50_000 / max(1.0, float(deg.sum()))))
    row_ptr, col_idx = sample_rows_pps(rng, deg, p)
    U0 = mean3_factors(rng, n_u, n_f)
    V0 = mean3_factors(rng, n_m, n_f)
    val = (low_rank_values(U0, V0, row_ptr, col_idx)
           + rng.normal(0.0, 0.5, size=len(col_idx))).astype(np.float32)
    return Problem("c3_batched", n_u, n_m, n_f, row_ptr, col_idx, val, 0.05,
                   budget[0], budget[1], 1, 15, init_factors(m0_seed, n_m, n_f), U0, V0, p)


def c4_precision(scale: float = 1.0, seed: int = 401, m0_seed: int = 402,
                 lam: float = 1e-4, budget=(1, 1)) -> Problem:
    """Precision sweep: 200k x 50k, n_f = 128, 2e7 uniform entries, ground truth
    with singular values log-spaced 1..1e3, no noise."""
    n_u = max(16, int(round(200_000 * scale)))
    n_m = max(16, int(round(50_000 * scale)))
    n_f = 128
    nnz = int(round(2e7 * scale))
    rng = np.random.default_rng(seed)
    keys = np.unique(rng.integers(0, n_u * n_m, size=int(nnz * 1.02) + 16, dtype=np.int64))
    if len(keys) > nnz:
        keys = np.sort(rng.choice(keys, size=nnz, replace=False))
    rows = keys // n_m
    cols = (keys % n_m).astype(np.int32)
    row_ptr = np.zeros(n_u + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n_u), out=row_ptr[1:])
    sig = 10.0 ** (3.0 * np.arange(n_f) / max(1, n_f - 1))
    Qu, _ = np.linalg.qr(rng.standard_normal((n_u, n_f)))
    Qv, _ = np.linalg.qr(rng.standard_normal((n_m, n_f)))
    c = (n_u * n_m / np.sum(sig ** 2)) ** 0.25
    U0 = c * Qu * np.sqrt(sig)[None, :]
    V0 = c * Qv * np.sqrt(sig)[None, :]
    val = low_rank_values(U0, V0, row_ptr, cols).astype(np.float32)
    return Problem("c4_precision", n_u, n_m, n_f, row_ptr, cols, val, lam,
                   budget[0], budget[1], 1, 10, init_factors(m0_seed, n_m, n_f), U0, V0)


def section5_factors(rng: np.random.Generator, n: int, n_f: int, dist: str) -> np.ndarray:
    """Factor rows of the simulation study (Section 5.1): D1 multivariate
    normal N(0, S), D2 multivariate log-normal LN(0, S) = exp of D1, D3
    multivariate t with 4 degrees of freedom, with S_ij = 0.6^|i - j|."""
    idx = np.arange(n_f)
    S = 0.6 ** np.abs(idx[:, None] - idx[None, :])
    Z = rng.standard_normal((n, n_f)) @ np.linalg.cholesky(S).T
    if dist == "D1":
        return Z
    if dist == "D2":
        return np.exp(Z)
    if dist == "D3":
        return Z / np.sqrt(rng.chisquare(4.0, size=(n, 1)) / 4.0)
    raise ValueError(dist)


def section5(dist: str = "D1", n_u: int = 5000, n_m: int = 5000, n_f: int = 50, alpha: float = 0.5,
             lam: float = 0.05, seed: int = 601, m0_seed: int = 602, n_heldout: int = 1_000_000):
    """The simulation workload of Section 5.1: R0 = U M^T from D1/D2/D3 factors,
    N(0, 1) noise on every entry, a fraction alpha of the entries observed
    (the rest, the prediction set I^c, set to NaN in the paper).  Returns the
    observed problem and a uniform sample of held-out entries (CSR over the
    same users) for the prediction error P-ReMSE."""
    rng = np.random.default_rng(seed)
    U0 = section5_factors(rng, n_u, n_f, dist)
    V0 = section5_factors(rng, n_m, n_f, dist)
    mask = rng.random((n_u, n_m)) < alpha
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(n_u + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n_u), out=row_ptr[1:])
    col_idx = cols.astype(np.int32)
    val = (low_rank_values(U0, V0, row_ptr, col_idx) + rng.normal(0.0, 1.0, size=len(col_idx))).astype(np.float32)
    prob = Problem(f"section5_{dist}", n_u, n_m, n_f, row_ptr, col_idx, val, lam, 1, 10, 1, 10,
                   init_factors(m0_seed, n_m, n_f), U0, V0)
    hr, hc = np.nonzero(~mask)
    if len(hr) > n_heldout:
        pick = np.sort(rng.choice(len(hr), size=n_heldout, replace=False))
        hr, hc = hr[pick], hc[pick]
    h_ptr = np.zeros(n_u + 1, dtype=np.int64)
    np.cumsum(np.bincount(hr, minlength=n_u), out=h_ptr[1:])
    h_idx = hc.astype(np.int32)
    h_val = (low_rank_values(U0, V0, h_ptr, h_idx) + rng.normal(0.0, 1.0, size=len(h_idx))).astype(np.float32)
    return prob, (h_ptr, h_idx, h_val)


def c5_heldout(base: Problem, n_new: int, seed: int = 502):
    """New users for fold-in: fresh user factors, the item side of `base`,
    degrees from the same Lomax law, values UV' + N(0, 0.25)."""
    rng = np.random.default_rng(seed)
    dmax = min(50_000, base.n_m)
    lscale = c3_scale_lomax(base.n_u, 1.0e8 * base.n_u / 1_000_000, 1.5, dmax)
    deg = lomax_degrees(rng, n_new, 1.5, lscale, dmax)
    p = base.item_p if base.item_p is not None else np.full(base.n_m, 1.0 / base.n_m)
    row_ptr, col_idx = sample_rows_pps(rng, deg, p)
    U0 = mean3_factors(rng, n_new, base.n_f)
    V0 = base.V_true if base.V_true is not None else mean3_factors(rng, base.n_m, base.n_f)
    val = (low_rank_values(U0, V0, row_ptr, col_idx)
           + rng.normal(0.0, 0.5, size=len(col_idx))).astype(np.float32)
    return row_ptr, col_idx, val


def arrival_batches(n_total: int, seed: int = 503):
    """Uneven arrival batch sizes clip(round(LogNormal(6, 1.5)), 1, 16384)."""
    rng = np.random.default_rng(seed)
    out = []
    left = n_total
    while left > 0:
        b = int(np.clip(np.round(rng.lognormal(6.0, 1.5)), 1, 16384))
        b = min(b, left)
        out.append(b)
        left -= b
    return out


def random_problem(seed: int, n_u: int, n_m: int, n_f: int, density: float,
                   lam: float = 0.05, budget=(1, 10), min_keep: int = 1,
                   rating_noise: float = 0.1, heavy_rows=()) -> Problem:
    """Small uniform-mask problem for tests; `heavy_rows` forces full rows."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n_u, n_m)) < density
    for r in heavy_rows:
        mask[r, :] = True
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(n_u + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n_u), out=row_ptr[1:])
    U0 = rng.normal(0.0, 1.0, size=(n_u, n_f)) / math.sqrt(n_f)
    V0 = rng.normal(0.0, 1.0, size=(n_m, n_f))
    val = low_rank_values(U0, V0, row_ptr, cols.astype(np.int32)) \
        + rng.normal(0.0, rating_noise, size=len(cols))
    M0 = rng.normal(0.0, 0.5, size=(n_m, n_f)).astype(np.float32)
    return Problem(f"random{seed}", n_u, n_m, n_f, row_ptr, cols.astype(np.int32),
                   val.astype(np.float32), lam, budget[0], budget[1], min_keep, 5, M0, U0, V0)


def foldin_init_params(seed: int, n_f: int, hidden: int) -> np.ndarray:
    """Seeded initial weights of the fold-in network, packed W1 [hidden x n_f],
    c1, W2 [hidden x hidden], c2, W3 [n_f x hidden], c3: weights uniform in
    +-1/sqrt(fan_in), biases zero (float32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((hidden, n_f), (hidden, hidden), (n_f, hidden)):
        lim = 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)
