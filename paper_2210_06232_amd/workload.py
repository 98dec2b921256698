"""The headline workload: one EI-FP step of a 256^3 grid on [0,2pi] x [0,4pi] x [0,2pi],
mu = eps = 1, tau = 0.1, seeded random divergence-free fields with spectrum
(1+|k|^2)^-2 cut at |k| <= 42.67 (the cut min_w(2 pi N_w / L_w)/3 of the recipe in
inputs.random_divfree)."""
from __future__ import annotations

import math

HEADLINE = {
    "workload": "eifp-maxwell-256^3-box[2pi,4pi,2pi]-mu1-eps1-tau0.1",
    "grid": [256, 256, 256],
    "domain": [0.0, 2 * math.pi, 0.0, 4 * math.pi, 0.0, 2 * math.pi],
    "mu": 1.0, "eps": 1.0, "tau": 0.1,
    "spectrum": "(1+|k|^2)^-2, 0<|k|<=42.67, transverse, seeded",
}


def headline_inputs():
    """(H, E) float64 [3, 256, 256, 256] each, seeded."""
    from . import inputs
    nx, ny, nz = HEADLINE["grid"]
    return inputs.random_fields((nx, ny, nz), tuple(HEADLINE["domain"]), workload=2, p=2.0)
