"""Performance regression gates on the 256^3 headline grid: the step time of both forms
and the bandwidth of the fused pass, with 30-40% margin over what one MI355X measures
(FP64 1.33-1.35 ms per step, fused pass 3.8 TB/s; FP32 0.70-0.71 ms, 3.3 TB/s), so that
a slow path (a kernel falling back to a worse configuration, a lost fusion) fails here
rather than only in the benchmark.  Inputs are white noise: the time does not depend on
them."""
import math
import time

import pytest

from paper_2210_06232_amd import inputs

pytestmark = pytest.mark.gpu

N = 256
BOX = (0.0, 2 * math.pi, 0.0, 4 * math.pi, 0.0, 2 * math.pi)
# form: (largest ms per step, smallest fused-pass GB/s of algorithmic traffic)
GATES = {"fp64": (1.9, 2900.0), "fp32": (1.0, 2300.0)}


@pytest.fixture(scope="module")
def fields():
    return inputs.white_noise_fields((N, N, N), 7)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_headline_step_time_and_fused_bandwidth(fields, prec):
    from paper_2210_06232_amd import eifp
    H, E = fields
    steps = 50
    with eifp.Solver(H, E, BOX, 1.0, 1.0, prec) as s:
        s.step(0.1, 5)
        s.sync()
        t0 = time.perf_counter()
        s.step(0.1, steps)
        s.sync()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        per = s.step_timed(0.1, steps)
    word = 8 if prec == "fp64" else 4
    fused_gbs = 2 * 6 * N ** 3 * word / (per["y_fused"] / steps * 1e-3) / 1e9
    max_ms, min_gbs = GATES[prec]
    assert ms <= max_ms, (prec, ms)
    assert fused_gbs >= min_gbs, (prec, fused_gbs)
