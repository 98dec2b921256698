"""Spatial convergence study of the scheme (Thm 3.4) on data of finite regularity.

The scheme is exact in time, so its whole error is spatial: a grid of N points per axis
carries the modes |k_w| < N/2 and aliases the rest.  The study draws one seeded,
divergence-free field pair whose Fourier amplitudes decay like (1+|k|^2)^-p up to the
reference grid's resolution (so the field has Sobolev regularity of about 2p - 3/2 and
the reference grid represents it exactly), samples it on coarser grids at the points
they share with the reference grid, advances every grid to t_end on the GPU in one
jump (FP64), and measures the relative energy-norm error at the shared points.  The
observed order is the slope of log(error) against log(N).

Run: python -m paper_2210_06232_amd.convergence --p 1.25,1.75 --nref 256 --ns 16,32,64,128
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

from . import eifp, inputs

TWO_PI = 2.0 * math.pi


def reference_fields(nref: int, p: float, domain, seed: int):
    """(H, E) on the nref^3 grid, every mode below the reference Nyquist radius kept."""
    L = (domain[1] - domain[0], domain[3] - domain[2], domain[5] - domain[4])
    kcut = min(TWO_PI * (nref // 2 - 1) / Lw for Lw in L)
    H = inputs.random_divfree((nref,) * 3, domain, seed, p=p, kcut=kcut)
    E = inputs.random_divfree((nref,) * 3, domain, seed + 1, p=p, kcut=kcut)
    return H, E


def subsample(F: np.ndarray, n: int) -> np.ndarray:
    """The values of a [3, N, N, N] field at the points of the n^3 grid (n divides N)."""
    s = F.shape[-1] // n
    return np.ascontiguousarray(F[:, ::s, ::s, ::s])


def energy_error(H, E, Hr, Er, mu, eps) -> float:
    num = mu * np.sum((H - Hr) ** 2) + eps * np.sum((E - Er) ** 2)
    den = mu * np.sum(Hr ** 2) + eps * np.sum(Er ** 2)
    return math.sqrt(num / den)


def run(p: float, nref: int, ns, t_end: float = 1.0, mu: float = 1.0, eps: float = 1.5, seed: int = 7000):
    domain = (0.0, TWO_PI, 0.0, TWO_PI, 0.0, TWO_PI)
    H0, E0 = reference_fields(nref, p, domain, seed)
    with eifp.Solver(H0, E0, domain, mu, eps, "fp64") as s:
        s.jump(t_end, 1)
        Hr, Er = s.fields()
    rows = []
    for n in ns:
        with eifp.Solver(subsample(H0, n), subsample(E0, n), domain, mu, eps, "fp64") as s:
            s.jump(t_end, 1)
            H, E = s.fields()
        rows.append({"n": n, "error": energy_error(H, E, subsample(Hr, n), subsample(Er, n), mu, eps)})
    for a, b in zip(rows, rows[1:]):
        b["order"] = math.log(a["error"] / b["error"]) / math.log(b["n"] / a["n"])
    return {"p": p, "nref": nref, "t_end": t_end, "mu": mu, "eps": eps, "rows": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--p", default="1.25,1.75")
    ap.add_argument("--nref", type=int, default=256)
    ap.add_argument("--ns", default="16,32,64,128")
    ap.add_argument("--t-end", type=float, default=1.0)
    a = ap.parse_args()
    for p in (float(x) for x in a.p.split(",")):
        print(json.dumps(run(p, a.nref, [int(x) for x in a.ns.split(",")], a.t_end)), flush=True)


if __name__ == "__main__":
    main()
