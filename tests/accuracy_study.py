"""Accuracy over long runs: the error of FP64 and FP32 stepping and of FP32 jumps
against the oracle, every `every` steps, with the drift of the energy and helicity.

Workload (the 64^3 companion of the 256^3 headline run): grid 64^3 on
[0,2pi] x [0,4pi] x [0,2pi], mu = eps = 1, tau = 0.1, seeded random divergence-free
fields with amplitudes (1+|k|^2)^-2.  The reference at step n is the oracle's single
step of n tau from the same input (the scheme is exact in time, so stepping and one
jump agree up to rounding).

Run: python tests/accuracy_study.py --steps 2000 --every 100
     python tests/accuracy_study.py --preset 1     (128^3, FP64, 1000 steps, every 100)
It lives with the tests because it uses the oracle as its reference.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2210_06232_amd import eifp, inputs  # noqa: E402

BOX = (0.0, 2 * math.pi, 0.0, 4 * math.pi, 0.0, 2 * math.pi)


def rel_err(H, E, Hr, Er, mu, eps) -> float:
    num = mu * np.sum((H - Hr) ** 2) + eps * np.sum((E - Er) ** 2)
    den = mu * np.sum(Hr ** 2) + eps * np.sum(Er ** 2)
    return math.sqrt(num / den)


def run(n: int = 64, steps: int = 2000, every: int = 100, tau: float = 0.1, mu: float = 1.0, eps: float = 1.0):
    H0, E0 = inputs.random_fields((n, n, n), BOX, workload=2, p=2.0)
    return study(H0, E0, BOX, mu, eps, tau, steps, every, ("fp64_step", "fp32_step", "fp32_jump"))


def run_preset(i: int, steps=None):
    """The same study on a named preset (its inputs, box, mu, eps, tau, step count and
    output interval), FP64 stepping only."""
    from paper_2210_06232_amd import workload
    cfg = workload.PRESETS[i]
    H0, E0 = workload.preset_inputs(cfg)
    return study(H0, E0, tuple(cfg["domain"]), cfg["mu"], cfg["eps"], cfg["tau"], steps or cfg["steps"],
                 cfg["every"], ("fp64_step",))


def study(H0, E0, box, mu, eps, tau, steps, every, forms):
    from oracle import oracle as orc
    solvers = {name: eifp.Solver(H0, E0, box, mu, eps, name.split("_")[0]) for name in forms}
    inv0 = {k: s.invariants() for k, s in solvers.items()}
    rows = []
    try:
        for k in range(every, steps + 1, every):
            Ho, Eo, _ = orc.step(H0, E0, box, mu, eps, tau * k, 1)
            row = {"step": k}
            for name, s in solvers.items():
                (s.jump if name.endswith("jump") else s.step)(tau, every)
                H, E = s.fields()
                inv = s.invariants()
                row[name] = rel_err(H, E, Ho, Eo, mu, eps)
                row[name + "_dE"] = (inv["energy"] - inv0[name]["energy"]) / inv0[name]["energy"]
                row[name + "_dH"] = inv["helicity"] - inv0[name]["helicity"]
            rows.append(row)
            print(json.dumps(row), flush=True)
    finally:
        for s in solvers.values():
            s.close()
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--preset", type=int, default=None, help="a named preset (its own sizes and steps)")
    a = ap.parse_args()
    if a.preset is not None:
        run_preset(a.preset)
    else:
        run(a.n, a.steps, a.every)


if __name__ == "__main__":
    main()
