"""Schedule autotuner for the half-sweep kernels.

The library's schedule has three knobs that depend on the degree distribution
of the matrix and on the GPU:

  heavy_min_degree  rows above this degree (or with budget > 32) are split
                    across workgroups instead of one wavefront per row;
  heavy_chunk       entries per partial Gram of a split row;
  light_blocks      grid of the persistent light-row kernels (0 = one row per
                    wavefront, no reuse of wavefronts).

The tuner times whole sweeps (users + items half-sweep, HIP-graph replay) on
the problem itself, coordinate by coordinate, and stores the best setting in
a JSON cache keyed by GPU architecture, n_f, precision, budget and a coarse
signature of the two degree distributions.  Timing uses HIP events on the
context's stream.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning", "gfx950.json")

DEFAULT = {"heavy_min_degree": 1024, "heavy_chunk": 1024, "light_blocks": 0}
SPACE = {
    "heavy_min_degree": [128, 192, 256, 384, 512, 1024, 2048],
    "heavy_chunk": [512, 1024, 2048, 4096],
    "light_blocks": [0, 1024, 2048, 4096],
}


def degree_signature(row_ptr: np.ndarray, col_idx: np.ndarray, n_cols: int) -> str:
    """Shares of rows and of entries per power-of-two degree bucket, both sides."""
    parts = []
    for deg in (np.diff(row_ptr), np.bincount(col_idx, minlength=n_cols)):
        b = np.floor(np.log2(np.maximum(deg, 1))).astype(int)
        rows = np.bincount(b, minlength=17)[:17] / max(1, len(deg))
        ents = np.bincount(b, weights=deg, minlength=17)[:17] / max(1, deg.sum())
        parts.append(",".join(f"{x:.2f}" for x in np.concatenate([rows, ents])))
    return "|".join(parts)


def cache_key(arch: str, n_f: int, precision: int, budget, sig: str, nnz: int) -> str:
    return f"{arch};nf={n_f};prec={precision};r={budget[0]}/{budget[1]};nnz~1e{math.log10(max(nnz, 1)):.1f};{sig}"


def load_cache(path: str = CACHE) -> Dict[str, dict]:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(cache: Dict[str, dict], path: str = CACHE) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_config(torch, prob, gpu_csr, budget, precision, cfg, stream, sweeps=2) -> float:
    """Milliseconds per sweep of one schedule setting (graph replay)."""
    from .als import CoreALS
    rp, ci, v = gpu_csr
    with torch.cuda.stream(stream):
        als = CoreALS(prob.n_u, prob.n_m, prob.n_f, rp, ci, v, prob.lam, budget, prob.min_keep,
                      precision, validate=False, stream=stream, graphs=True, **cfg)
        M = torch.from_numpy(prob.M0).to(rp.device)
        U = torch.empty(prob.n_u, prob.n_f, dtype=torch.float32, device=rp.device)
        # three untimed sweeps: the heavy-row selection starts from the
        # previous sweep's cuts once the factors have settled a little
        for _ in range(3):
            als.half_sweep_users(M, U)
            als.half_sweep_items(U, M)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(sweeps):
            als.half_sweep_users(M, U)
            als.half_sweep_items(U, M)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / sweeps
        als.close()
    return ms


def tune(torch, prob, gpu_csr, budget, precision, stream=None, log=None, path: Optional[str] = CACHE,
         force: bool = False) -> dict:
    """Best schedule for this problem: cached if known, else a coordinate search."""
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    sig = degree_signature(prob.row_ptr, prob.col_idx, prob.n_m)
    key = cache_key(arch, prob.n_f, precision, budget, sig, prob.nnz)
    cache = load_cache(path) if path else {}
    if not force and key in cache:
        if log:
            log(f"autotune: cached {cache[key]['config']}")
        return dict(cache[key]["config"])
    stream = stream or torch.cuda.Stream()
    best = dict(DEFAULT)
    best_ms = time_config(torch, prob, gpu_csr, budget, precision, best, stream)
    trials = [(dict(best), best_ms)]
    t0 = time.time()
    # two rounds of coordinate descent: the best degree limit depends on the
    # grid of the light-row kernels and the other way round
    for knob in ("heavy_min_degree", "heavy_chunk", "light_blocks") * 2:
        for val in SPACE[knob]:
            if val == best[knob]:
                continue
            cfg = dict(best)
            cfg[knob] = val
            ms = time_config(torch, prob, gpu_csr, budget, precision, cfg, stream)
            trials.append((cfg, ms))
            if log:
                log(f"autotune r={budget[0]}/{budget[1]} precision {precision}: {cfg} {ms:.2f} ms/sweep")
            if ms < best_ms:
                best, best_ms = cfg, ms
    if log:
        log(f"autotune: {len(trials)} settings in {time.time() - t0:.1f}s, best {best} at {best_ms:.2f} ms/sweep")
    if path:
        cache[key] = {"config": best, "ms_per_sweep": best_ms,
                      "trials": [{"config": c, "ms": m} for c, m in trials]}
        save_cache(cache, path)
    return best
