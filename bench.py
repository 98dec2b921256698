#!/usr/bin/env python3
"""Benchmark of the EI-FP time step on one MI355X.

A step is one pass of the whole hot path over the state: forward 3-D FFT of the six
field components (x R2C, y, z), the exact mode-wise propagator, the invariant partial
sums, the inverse FFT (z, y, x C2R) and the deterministic invariant finalize.

Workload: 256^3 grid on [0,2pi] x [0,4pi] x [0,2pi], mu = eps = 1, tau = 0.1, seeded
random divergence-free fields with spectrum (1+|k|^2)^-2 cut at |k| <= 42.67.  Fields
are uploaded before the timed region (the state is resident in HBM).

Prints ONE JSON line.  ``value`` is FP64 field-point-steps/s; the FP32 form is timed on
the same input and reported under ``"fp32"``.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
WORKLOAD = {
    "workload": "eifp-maxwell-256^3-box[2pi,4pi,2pi]-mu1-eps1-tau0.1",
    "grid": [256, 256, 256],
    "domain": [0.0, 2 * math.pi, 0.0, 4 * math.pi, 0.0, 2 * math.pi],
    "mu": 1.0, "eps": 1.0, "tau": 0.1,
    "spectrum": "(1+|k|^2)^-2, 0<|k|<=42.67, transverse, seeded",
}
PASSES = ("x_fwd", "z_fwd", "y_fused", "z_inv", "x_inv", "finalize")
KERNEL_NAMES = {"x_fwd": "k_x_fwd", "z_fwd": "k_c2c", "y_fused": "k_fused", "z_inv": "k_c2c",
                "x_inv": "k_x_inv", "finalize": "k_finalize"}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2210_06232_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".h", ".hip")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(prec: str, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic_256cubed.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
        if rec.get("source_hash") != kernel_source_hash():
            return None
        ent = rec["kernels"][prec][kernel]
        return float(ent["fetch_bytes"]) + float(ent["write_bytes"])
    except (KeyError, ValueError, TypeError):
        return None


def make_inputs():
    from paper_2210_06232_amd import inputs
    nx, ny, nz = WORKLOAD["grid"]
    return inputs.random_fields((nx, ny, nz), tuple(WORKLOAD["domain"]), workload=2, p=2.0)


def run_gpu(H, E, prec: str, steps: int, warmup: int):
    import torch
    from paper_2210_06232_amd import eifp
    nx, ny, nz = WORKLOAD["grid"]
    ns = nx * ny * nz
    tsize = 8 if prec == "fp64" else 4
    with eifp.Solver(H, E, WORKLOAD["domain"], WORKLOAD["mu"], WORKLOAD["eps"], prec) as s:
        if warmup:
            s.step(WORKLOAD["tau"], warmup)
        s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pass_ms = s.step_timed(WORKLOAD["tau"], steps)   # events on the solver's stream; syncs
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        inv = s.invariants()
    ms_per_step = 1e3 * wall / steps
    per_launch = {k: v / steps for k, v in pass_ms.items()}
    dominant = max(PASSES[:5], key=lambda k: per_launch[k])
    # algorithmic bytes per launch of any of the five passes: read and write the whole
    # state once (6 components x N_S reals)
    alg_bytes = 2.0 * 6 * ns * tsize
    achieved = alg_bytes / (per_launch[dominant] * 1e-3) / 1e9
    traffic = measured_traffic(prec, dominant)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                "kernel": KERNEL_NAMES[dominant], "pass": dominant,
                "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": round(per_launch[dominant], 5)}
    step_bw = 5 * alg_bytes / (ms_per_step * 1e-3) / 1e9
    return {
        "value": ns / (ms_per_step * 1e-3),
        "ms_per_step": ms_per_step,
        "pass_ms_per_step": {k: round(v, 5) for k, v in per_launch.items()},
        "roofline": roofline,
        "step_hbm_gbs_5pass_model": round(step_bw, 1),
        "energy": inv["energy"],
    }


def cpu_baseline(H, E):
    """The FP64 CPU oracle as it stands, one step of the same 256^3 workload, one thread."""
    from oracle import oracle as orc
    nx, ny, nz = WORKLOAD["grid"]
    t0 = time.perf_counter()
    orc.step(H, E, WORKLOAD["domain"], WORKLOAD["mu"], WORKLOAD["eps"], WORKLOAD["tau"], 1)
    dt = time.perf_counter() - t0
    return {"value": nx * ny * nz / dt, "unit": "field-point-steps/s", "cores": 1, "kind": "oracle",
            "sample": "1 step of the 256^3 workload (full grid), FP64, single thread",
            "seconds": round(dt, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(value is the one GPU's throughput)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    H, E = make_inputs()
    print(f"[bench] inputs ready {H.shape}", file=sys.stderr, flush=True)
    r64 = run_gpu(H, E, "fp64", args.steps, args.warmup)
    print(f"[bench] fp64 {r64['ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)
    r32 = run_gpu(H, E, "fp32", args.steps, args.warmup)
    print(f"[bench] fp32 {r32['ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)
    cpu = None
    if rank == 0 and not args.no_cpu_baseline:
        cpu = cpu_baseline(H, E)
        print(f"[bench] cpu oracle {cpu['seconds']} s/step", file=sys.stderr, flush=True)

    out = {
        "metric": "field-point-steps/s at 256^3 FP64 vs FP32 (% HBM roofline)",
        "value": r64["value"],
        "unit": "field-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": WORKLOAD,
        "roofline": r64["roofline"],
        "cpu_baseline": cpu,
        "pass_ms_per_step": r64["pass_ms_per_step"],
        "fp32": {"value": r32["value"], "ms_per_step": r32["ms_per_step"], "dtype": "f32",
                 "roofline": r32["roofline"], "pass_ms_per_step": r32["pass_ms_per_step"]},
        "kernel_source_hash": kernel_source_hash(),
    }
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
