"""The workloads: the headline one (one EI-FP step of a 256^3 grid on [0,2pi] x [0,4pi]
x [0,2pi], mu = eps = 1, tau = 0.1, seeded random divergence-free fields with spectrum
(1+|k|^2)^-2 cut at |k| <= 42.67, the cut min_w(2 pi N_w / L_w)/3 of the recipe in
inputs.random_divfree), and named presets of the others with a runner that reports
their point-step rate and the drift of every invariant
(python -m paper_2210_06232_amd.workload --preset i)."""
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


# ---------------------------------------------------------------------------------
# named presets of the other workloads, and a runner that reports their point-step
# rate and the drift of the invariants (python -m paper_2210_06232_amd.workload)
# ---------------------------------------------------------------------------------
CUBE = [0.0, 2 * math.pi, 0.0, 2 * math.pi, 0.0, 2 * math.pi]
PRESETS = {
    0: {"workload": "standing-wave-16^3-mu1-eps1-tau0.01", "grid": [16, 16, 16], "domain": CUBE,
        "mu": 1.0, "eps": 1.0, "tau": 0.01, "steps": 100, "every": 10, "precs": ["fp64"], "fields": "standing",
        "t0": [0.0, 0.3]},
    1: {"workload": "random-divfree-128^3-mu1-eps2-tau0.05", "grid": [128, 128, 128], "domain": CUBE,
        "mu": 1.0, "eps": 2.0, "tau": 0.05, "steps": 1000, "every": 100, "precs": ["fp64"], "p": 2.0, "seed": 1},
    2: {**HEADLINE, "steps": 2000, "every": 100, "precs": ["fp64", "fp32"], "p": 2.0, "seed": 2},
    3: {"workload": "random-divfree-512^3-mu1-eps1.5-tau0.02", "grid": [512, 512, 512], "domain": CUBE,
        "mu": 1.0, "eps": 1.5, "tau": 0.02, "steps": 10000, "every": 1000, "precs": ["fp32"], "p": 1.5, "seed": 3},
}


def preset_inputs(cfg, progress=None, t0=0.0, cache=None):
    """(H, E) float64 [3, nz, ny, nx] of a preset: the standing wave at t = 0 (phase
    offset t0), or the seeded random divergence-free fields of inputs.random_fields
    (about a minute per field at 512^3 on one core).  With cache (a directory), the
    random fields are loaded from cache/<workload>_{H,E}.npy when present and saved
    there after generation otherwise."""
    import os
    import numpy as np
    from . import inputs
    nx, ny, nz = cfg["grid"]
    if cfg.get("fields") == "standing":
        H, E, _ = inputs.standing_wave(nx, 0.0, cfg["mu"], cfg["eps"], t0)
        return H, E
    paths = [os.path.join(cache, f"{cfg['workload']}_{c}.npy") for c in "HE"] if cache else None
    if paths and all(os.path.exists(q) for q in paths):
        if progress:
            progress(f"{cfg['workload']}: loading cached fields")
        return tuple(np.load(q) for q in paths)
    fields = []
    for part in range(2):
        if progress:
            progress(f"{cfg['workload']}: generating field {'HE'[part]}")
        fields.append(inputs.random_divfree((nx, ny, nz), tuple(cfg["domain"]),
                                            inputs.SEED_BASE + 1000 * cfg["seed"] + part, p=cfg["p"]))
    if paths:
        os.makedirs(cache, exist_ok=True)
        for q, a in zip(paths, fields):
            np.save(q, a)
    return tuple(fields)


def _rel(d, scale):
    """A drift relative to its scale; the raw drift where the scale is zero (the
    invariant is then zero at every step up to rounding)."""
    return d / scale if scale > 0 else d


def run_preset(i: int, steps=None, precs=None, progress=None, cache=None):
    """Step preset i in chunks of cfg['every'] steps; returns, per precision (and per
    phase offset t0 of the standing wave), the field-point-steps/s of the stepping
    (device-synchronised, readbacks excluded) and the drift of every invariant after each
    chunk: the energy relative to its initial value, helicity, momentum and divergence
    norms relative to their drift scales; the energy's least-squares slope in unit
    roundoffs of the precision per step; for the standing wave the error against the
    exact solution."""
    from . import eifp
    cfg = PRESETS[i]
    steps = steps or cfg["steps"]
    every = min(cfg["every"], steps)
    dom = tuple(cfg["domain"])
    out = {"preset": i, "workload": cfg["workload"], "steps": steps, "every": every, "runs": {}}
    t0s = cfg.get("t0", [0.0])
    for t0 in t0s:
        H, E = preset_inputs(cfg, progress, t0, cache)
        for prec in precs or cfg["precs"]:
            label = prec if len(t0s) == 1 else f"{prec}_t0={t0:g}"
            with eifp.Solver(H, E, dom, cfg["mu"], cfg["eps"], prec) as warm:
                warm.step(cfg["tau"], every)  # first launches of this shape stay out of the timing
                warm.sync()
            s = eifp.Solver(H, E, dom, cfg["mu"], cfg["eps"], prec)
            try:
                out["runs"][label] = _run_one(s, cfg, steps, every, t0, prec, progress, f"preset {i} {label}")
            finally:
                s.close()
    return out


def _run_one(s, cfg, steps, every, t0, prec, progress, name):
    import time
    from . import inputs
    nx, ny, nz = cfg["grid"]
    i0, x0 = s.invariants(), s.invariants_ext()
    t_step, done, rows = 0.0, 0, []
    while done < steps:
        n = min(every, steps - done)
        s.sync()
        t0_ = time.perf_counter()
        s.step(cfg["tau"], n)
        s.sync()
        t_step += time.perf_counter() - t0_
        done += n
        inv = s.invariants()
        rows.append({
            "step": done,
            "energy": (inv["energy"] - i0["energy"]) / i0["energy"],
            "helicity": _rel(inv["helicity"] - i0["helicity"], x0["scale_helicity"]),
            "momentum": max((_rel(inv["momentum"][k] - i0["momentum"][k], x0["scale_momentum"][k])
                             for k in range(3)), key=abs),
            "div_h": _rel(inv["div_h_l2"] - i0["div_h_l2"], x0["scale_div_h"]),
            "div_e": _rel(inv["div_e_l2"] - i0["div_e_l2"], x0["scale_div_e"])})
        if progress:
            progress(f"{name}: {done}/{steps} steps")
    u = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24
    slope = sum(r["step"] * r["energy"] for r in rows) / sum(r["step"] ** 2 for r in rows)
    run = {"point_steps_per_s": nx * ny * nz * steps / t_step, "ms_per_step": 1e3 * t_step / steps,
           "max_abs_drift": {k: max(abs(r[k]) for r in rows) for k in rows[0] if k != "step"},
           "energy_slope_u_per_step": slope / u, "drift": rows}
    if cfg.get("fields") == "standing":
        Hx, Ex, _ = inputs.standing_wave(nx, cfg["tau"] * steps, cfg["mu"], cfg["eps"], t0)
        Hg, Eg = s.fields()
        num = cfg["mu"] * float(((Hg - Hx) ** 2).sum()) + cfg["eps"] * float(((Eg - Ex) ** 2).sum())
        den = cfg["mu"] * float((Hx ** 2).sum()) + cfg["eps"] * float((Ex ** 2).sum())
        run["rel_error_vs_exact"] = math.sqrt(num / den)
    return run


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="run a named workload preset")
    ap.add_argument("--preset", type=int, required=True, choices=sorted(PRESETS))
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--prec", default=None, help="comma list (default: the preset's)")
    ap.add_argument("--inputs-cache", default=None, help="directory for the generated random fields")
    a = ap.parse_args()
    res = run_preset(a.preset, a.steps, a.prec.split(",") if a.prec else None,
                     progress=lambda msg: print(msg, flush=True), cache=a.inputs_cache)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
