"""The serving stream's request recipe (host only): grids from the fixed set, about
70% FP32, log-uniform step counts on [10, 5000], cadence on [10, 500], Poisson arrivals."""
import math

import numpy as np

from paper_2210_06232_amd import serving


def test_stream_recipe():
    reqs = serving.make_stream(4000, pool=8)
    assert {r["shape"] for r in reqs} == set(serving.STREAM_SHAPES)
    frac32 = np.mean([r["prec"] == "fp32" for r in reqs])
    assert abs(frac32 - 0.7) < 0.03
    ns = np.array([r["nsteps"] for r in reqs])
    assert ns.min() >= 10 and ns.max() <= 5000
    # log-uniform on [10, 5000]: mean (5000 - 10) / ln 500 = 803; median sqrt(10 * 5000) = 224
    assert abs(ns.mean() / ((5000 - 10) / math.log(500)) - 1) < 0.08
    assert abs(np.median(ns) / math.sqrt(10 * 5000) - 1) < 0.15
    cad = np.array([r["cadence"] for r in reqs])
    assert cad.min() >= 10 and cad.max() <= 500
    assert all(0.01 <= r["tau"] <= 0.1 and 1 <= r["eps"] <= 2 and r["mu"] == 1 for r in reqs)
    assert {r["pool_index"] for r in reqs} == set(range(8))
    box = [r for r in reqs if r["shape"] == (64, 128, 256)][0]["domain"]
    # the same spacing on every axis
    assert np.allclose([(box[1] - box[0]) / 64, (box[3] - box[2]) / 128, (box[5] - box[4]) / 256], 2 * math.pi / 64)
    # same seed, same stream
    assert serving.make_stream(50) == serving.make_stream(50)


def test_poisson_arrivals():
    reqs = serving.add_arrivals(serving.make_stream(5000), rate=20.0)
    t = np.array([r["arrival"] for r in reqs])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    assert abs(gaps.mean() * 20.0 - 1) < 0.05
    # exponential gaps: the coefficient of variation is 1
    assert abs(gaps.std() / gaps.mean() - 1) < 0.05
