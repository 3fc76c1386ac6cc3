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
