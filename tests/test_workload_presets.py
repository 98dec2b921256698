"""The named workload presets: their table (host), and a short run of the small ones
on the GPU — the 16^3 standing wave against its exact solution, the 128^3 random
fields for the conservation of every invariant over the run."""
import math

import numpy as np
import pytest

from paper_2210_06232_amd import inputs, workload


def test_preset_table():
    for i, cfg in workload.PRESETS.items():
        for key in ("workload", "grid", "domain", "mu", "eps", "tau", "steps", "every", "precs"):
            assert key in cfg, (i, key)
        assert cfg["steps"] % cfg["every"] == 0
        assert set(cfg["precs"]) <= {"fp64", "fp32"}
    assert workload.PRESETS[2]["grid"] == workload.HEADLINE["grid"]
    assert workload.PRESETS[2]["workload"] == workload.HEADLINE["workload"]


def test_headline_preset_inputs_are_the_headline_inputs():
    # same recipe, same seeds: generated at 32^3 through both paths
    cfg = dict(workload.PRESETS[2], grid=[32, 32, 32])
    H, E = workload.preset_inputs(cfg)
    Hr, Er = inputs.random_fields((32, 32, 32), tuple(cfg["domain"]), workload=2, p=2.0)
    assert np.array_equal(H, Hr) and np.array_equal(E, Er)


def test_standing_wave_preset_starts_at_rest_in_e():
    H, E = workload.preset_inputs(workload.PRESETS[0])
    assert H.shape == (3, 16, 16, 16) and not E.any()
    # normalised so that the discrete mean of |H|^2 is 1
    assert abs(float((H ** 2).sum()) / 16 ** 3 - 1.0) < 1e-13
    H3, E3 = workload.preset_inputs(workload.PRESETS[0], t0=0.3)
    assert E3.any() and not np.array_equal(H3, H)


def test_preset_input_cache_round_trip(tmp_path):
    cfg = dict(workload.PRESETS[1], grid=[8, 8, 8], workload="cache-probe-8^3")
    a = workload.preset_inputs(cfg, cache=str(tmp_path))
    assert sorted(p.name for p in tmp_path.iterdir()) == ["cache-probe-8^3_E.npy", "cache-probe-8^3_H.npy"]
    b = workload.preset_inputs(cfg, cache=str(tmp_path))
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.gpu
def test_standing_wave_preset_matches_exact_solution():
    # t0 = 0 (E starts at zero) and t0 = 0.3 (both fields non-zero)
    res = workload.run_preset(0)
    assert sorted(res["runs"]) == ["fp64_t0=0", "fp64_t0=0.3"]
    for run in res["runs"].values():
        assert run["rel_error_vs_exact"] <= 1e-12
        assert run["max_abs_drift"]["energy"] <= 1e-13
        assert run["point_steps_per_s"] > 0


@pytest.mark.gpu
def test_random_preset_conserves_every_invariant():
    res = workload.run_preset(1, steps=40, precs=["fp64", "fp32"])
    d64 = res["runs"]["fp64"]["max_abs_drift"]
    d32 = res["runs"]["fp32"]["max_abs_drift"]
    assert len(res["runs"]["fp64"]["drift"]) == 1  # 40 steps in one chunk of at most 100
    for k in ("energy", "helicity", "momentum", "div_h", "div_e"):
        assert math.isfinite(d64[k]) and d64[k] <= 1e-12, (k, d64[k])
        assert math.isfinite(d32[k]) and d32[k] <= 1e-4, (k, d32[k])
