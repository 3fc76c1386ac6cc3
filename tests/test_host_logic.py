"""Host-side logic that needs no GPU: schedule tuning cache, input generators."""
import json

import numpy as np

from paper_2509_18024_amd import autotune, synth


def test_degree_signature_and_cache_roundtrip(tmp_path):
    p = synth.random_problem(3, 200, 150, 8, 0.1, heavy_rows=(1,))
    sig = autotune.degree_signature(p.row_ptr, p.col_idx, p.n_m)
    assert sig == autotune.degree_signature(p.row_ptr.copy(), p.col_idx.copy(), p.n_m)
    key = autotune.cache_key("gfx950", 8, 1, (1, 10), sig, p.nnz)
    path = str(tmp_path / "t.json")
    autotune.save_cache({key: {"config": {"heavy_min_degree": 512}}}, path)
    assert autotune.load_cache(path)[key]["config"]["heavy_min_degree"] == 512
    json.load(open(path))


def test_committed_tuning_cache_is_well_formed():
    cache = autotune.load_cache()
    for key, entry in cache.items():
        assert key.startswith("gfx950;")
        assert set(entry["config"]) == set(autotune.DEFAULT)
        for knob, val in entry["config"].items():
            assert val in autotune.SPACE[knob]


def test_generators_are_seeded_and_rows_sorted():
    a = synth.c2_core(scale=0.01)
    b = synth.c2_core(scale=0.01)
    assert np.array_equal(a.col_idx, b.col_idx) and np.array_equal(a.val, b.val)
    r = synth.rows_of(a.row_ptr)
    assert np.all((r[1:] != r[:-1]) | (a.col_idx[1:] > a.col_idx[:-1]))
    assert a.val.min() >= 1 and a.val.max() <= 5 and np.all(a.val == np.round(a.val))


def test_pps_sampling_gives_exact_distinct_degrees():
    rng = np.random.default_rng(0)
    deg = np.array([1, 5, 50, 300, 900, 1000])
    p = synth.zipf_weights(rng, 1000, 1.1)
    rp, ci = synth.sample_rows_pps(rng, deg, p / p.sum())
    assert np.array_equal(np.diff(rp), deg)
    for i in range(len(deg)):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)


def test_c3_small_scale_shape():
    p = synth.c3_batched(scale=0.002)
    d = np.diff(p.row_ptr)
    assert p.n_f == 64 and d.min() >= 1 and p.nnz > 0.8e8 * 0.002


def test_binding_constants_match_the_header():
    """The ctypes binding repeats the C header's enum values and flag bits; a
    mismatch would pass wrong flags or misread status codes."""
    import os
    import re
    from paper_2509_18024_amd import capi
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "include", "coreals.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    defines = dict((k, int(v)) for k, v in re.findall(r"#define\s+(ALS_\w+)\s+(\d+)u?\b", text))
    enums = dict((k, int(v)) for k, v in re.findall(r"\b(ALS_\w+|FOLDIN_\w+)\s*=\s*(\d+)", text))
    assert {"ALS_VALIDATE", "ALS_USERS_ONLY", "ALS_GENERIC_GATHERS"} <= set(defines)
    assert {"ALS_OK", "ALS_E_STATE", "ALS_PREC_FP32", "ALS_PREC_AUTO"} <= set(enums)
    flags = [defines[k] for k in ("ALS_VALIDATE", "ALS_USERS_ONLY", "ALS_GENERIC_GATHERS")]
    assert all(f & (f - 1) == 0 for f in flags) and len(set(flags)) == len(flags)  # distinct bits
    for name, value in {**defines, **enums}.items():
        if hasattr(capi, name):
            assert getattr(capi, name) == value, name
    for name in ("ALS_VALIDATE", "ALS_USERS_ONLY", "ALS_GENERIC_GATHERS", "ALS_OK", "ALS_E_ARG",
                 "ALS_E_STATE", "ALS_PREC_FP32", "ALS_PREC_BF16_IR", "ALS_PREC_AUTO"):
        assert hasattr(capi, name), name


def _counter_csv(path, rows):
    """A rocprofv3 counter_collection.csv with the columns the digest reads."""
    import csv
    path.mkdir(parents=True, exist_ok=True)
    with open(path / "x_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, k, c, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_traffic_digest_scales_by_the_copy_kernel(tmp_path):
    """The copy kernel moves 1 GiB each way; its readings fix one factor per
    counter, and a kernel's bytes per launch are the means of its dispatches
    after the skipped ones, each counter times its factor."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    kib = float(1 << 20)  # 1 GiB in KiB
    ew = "void at::native::elementwise_kernel<...>"
    _counter_csv(tmp_path / "cf", [(1, ew, "FETCH_SIZE", kib / 2), (2, ew, "FETCH_SIZE", kib / 2)])  # factor 2
    _counter_csv(tmp_path / "cw", [(1, ew, "WRITE_SIZE", kib)])                                      # factor 1
    k = "void coreals::k_heavy_select<true, true>(coreals::HeavyArgs, long)"
    _counter_csv(tmp_path / "f", [(1, k, "FETCH_SIZE", 999.0), (3, k, "FETCH_SIZE", 100.0),
                                  (5, k, "FETCH_SIZE", 300.0)])
    _counter_csv(tmp_path / "w", [(1, k, "WRITE_SIZE", 999.0), (3, k, "WRITE_SIZE", 10.0),
                                  (5, k, "WRITE_SIZE", 30.0)])
    out = tmp_path / "digest.json"
    subprocess.run([sys.executable, os.path.join(root, "paper_2509_18024_amd", "tuning", "traffic_digest.py"),
                    "--fetch", str(tmp_path / "f"), "--write", str(tmp_path / "w"),
                    "--copy-fetch", str(tmp_path / "cf"), "--copy-write", str(tmp_path / "cw"),
                    "--skip", "1", "--kernels", "k_heavy_select", "--out", str(out)],
                   check=True, stdout=subprocess.PIPE)
    d = json.load(open(out))
    assert d["fetch_factor"] == 2.0 and d["write_factor"] == 1.0
    e = d["kernels"]["k_heavy_select"]
    assert e["dispatches"] == 2
    assert e["fetch_bytes_per_launch"] == 200.0 * 1024 * 2.0   # mean of 100 and 300 KiB, doubled
    assert e["write_bytes_per_launch"] == 20.0 * 1024
    assert e["hbm_bytes_per_launch"] == e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]


def test_traffic_figure_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    import bench
    path = tmp_path / "t.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic("k_heavy_select") is None  # no digest
    entry = {"kernels": {"k_heavy_select": {"hbm_bytes_per_launch": 5.0}}}
    json.dump(dict(entry, source_sha256=bench.kernel_source_digest()), open(path, "w"))
    assert bench.measured_traffic("k_heavy_select") == 5.0
    assert bench.measured_traffic("k_heavy_gram_x6") is None
    json.dump(dict(entry, source_sha256="0" * 64), open(path, "w"))
    assert bench.measured_traffic("k_heavy_select") is None  # taken on other sources


def test_tuner_coordinate_search_and_cache(tmp_path, monkeypatch):
    """The schedule search with a synthetic cost (no GPU): two rounds of
    coordinate descent reach the cost's minimum, every trial is recorded, and
    a second call returns the cached setting without timing anything."""
    import types
    p = synth.random_problem(4, 120, 90, 8, 0.1)
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(
        get_device_properties=lambda i: types.SimpleNamespace(gcnArchName="gfx950:sramecc+:xnack-"),
        Stream=lambda: None))
    want = {"heavy_min_degree": 384, "heavy_chunk": 2048, "light_blocks": 1024}
    calls = []

    def cost(torch, prob, gpu_csr, budget, precision, cfg, stream, sweeps=2):
        calls.append(dict(cfg))
        # separable except for a coupling that a single round would miss
        c = sum(abs(autotune.SPACE[k].index(cfg[k]) - autotune.SPACE[k].index(want[k])) for k in want)
        return 10.0 + c + (0.5 if cfg["light_blocks"] == 0 and cfg["heavy_min_degree"] != 1024 else 0.0)

    monkeypatch.setattr(autotune, "time_config", cost)
    path = str(tmp_path / "cache.json")
    best = autotune.tune(fake_torch, p, None, (1, 10), 0, stream=object(), path=path)
    assert best == want
    entry = next(iter(autotune.load_cache(path).values()))
    assert entry["config"] == want and entry["ms_per_sweep"] == 10.0
    assert len(entry["trials"]) == len(calls)
    n = len(calls)
    assert autotune.tune(fake_torch, p, None, (1, 10), 0, stream=object(), path=path) == want
    assert len(calls) == n  # cached: nothing timed
