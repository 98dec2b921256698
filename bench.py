#!/usr/bin/env python3
"""Benchmark of the EI-FP time step on one MI355X, and of the serving loop.

A step is one pass of the whole hot path over the state: forward 3-D FFT of the six
field components (x R2C, z, y), the exact mode-wise propagator, the invariant partial
sums, the inverse FFT (y, z, x C2R) and the deterministic invariant finalize.  The
timed steps run as one call: between two steps the x inverse of one and the x forward
of the next are one kernel (k_x_invfwd), which keeps the intermediate physical state in
registers; the call's last step writes the state.

Workload: 256^3 grid on [0,2pi] x [0,4pi] x [0,2pi], mu = eps = 1, tau = 0.1, seeded
random divergence-free fields with spectrum (1+|k|^2)^-2 cut at |k| <= 42.67.  Fields
are uploaded before the timed region (the state is resident in HBM).

Serving: a seeded stream of mixed-size solves (7 grids from 32^3 to 256^3, 70% FP32,
log-uniform step counts on [10, 5000]) replayed against the batching server, once with
Poisson arrivals at 0.8 of one-at-a-time capacity (latency) and once with every
request arriving at once (throughput), each beside serial FP64 solves of the same
stream.

Prints ONE JSON line.  ``value`` is FP64 field-point-steps/s; the FP32 form is timed on
the same input and reported under ``"fp32"``; serving under ``"serving"``.  The same K
FP64 steps as a caller holding the fields in host memory sees them (init from host
arrays, the steps, the fields back to host arrays) are reported under ``"host_to_host"``,
beside ``value``, never as it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2210_06232_amd.profiling import kernel_source_hash  # noqa: E402
from paper_2210_06232_amd.workload import HEADLINE as WORKLOAD, headline_inputs  # noqa: E402

PEAK_HBM_GBS = 8000.0
PASSES = ("x_fwd", "z_fwd", "y_fused", "z_inv", "x_inv", "finalize")
# the x-inverse slot holds the combined x kernel (every step but the last) and one k_x_inv
KERNEL_NAMES = {"x_fwd": "k_x_fwd", "z_fwd": "k_c2c", "y_fused": "k_fused", "z_inv": "k_c2c",
                "x_inv": "k_x_invfwd", "finalize": "k_finalize"}


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


# Vector-ALU issue ceiling: 256 CUs x 4 SIMDs, one wave64 VALU instruction per SIMD every
# 4 cycles (16 lanes per clock, the FP64 and non-packed FP32 rate behind the 78.6 TFLOP/s
# FP64 vector peak: 256 x 4 x 16 x 2 flop x 2.4 GHz), at 2.4 GHz.
PEAK_VALU_GIPS = 256 * 4 * 2.4e9 / 4 / 1e9


def measured_valu(prec: str, kernel: str):
    """VALU wave-instructions per launch of the step's `kernel` from the committed SQ
    counter summary, if it was taken on the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", "step_256cubed_sq_counters.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
        if rec.get("source_hash") != kernel_source_hash():
            return None
        ctype = "double" if prec == "fp64" else "float"
        for name, ent in rec["kernels"].items():
            if name.startswith(f"{kernel}<{ctype},"):
                return float(ent["raw"]["SQ_INSTS_VALU"])
    except (KeyError, ValueError, TypeError):
        return None
    return None


def timed_steps(s, steps: int):
    """K steps of the headline workload on solver s, timed; returns (wall s, pass ms)."""
    import torch
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pass_ms = s.step_timed(WORKLOAD["tau"], steps)   # events on the solver's stream; syncs
    torch.cuda.synchronize()
    return time.perf_counter() - t0, pass_ms


def run_gpu_pair(H, E, steps: int, warmup: int):
    """Both forms on the same input.  Both solvers are created (their uploads done) before
    any step runs, and the device then stays busy from the first warmup step to the last
    timed one: W FP32 warmup steps, W FP64 warmup steps, K timed FP64 steps, K timed FP32
    steps.  After an idle gap (an upload) the compute clock needs ~20 ms to settle, which
    a few warmup steps alone would leave inside a short timed region."""
    from paper_2210_06232_amd import eifp
    args = (H, E, WORKLOAD["domain"], WORKLOAD["mu"], WORKLOAD["eps"])
    with eifp.Solver(*args, "fp64") as s64, eifp.Solver(*args, "fp32") as s32:
        for s in (s32, s64):
            if warmup:
                s.step(WORKLOAD["tau"], warmup)
                s.sync()  # one form at a time: the two solvers' streams never share the device
        t64 = timed_steps(s64, steps)
        t32 = timed_steps(s32, steps)
        inv64, inv32 = s64.invariants(), s32.invariants()
    return summarize("fp64", steps, *t64, inv64), summarize("fp32", steps, *t32, inv32)


def host_to_host(H, E, steps: int):
    """K FP64 steps from host arrays to host arrays: eifp_init (allocation, the
    non-finite check, upload and relayout), the steps, eifp_fields (download and
    relayout), timed from the host with the device idle before and synchronised after."""
    import torch
    from paper_2210_06232_amd import eifp
    nx, ny, nz = WORKLOAD["grid"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with eifp.Solver(H, E, WORKLOAD["domain"], WORKLOAD["mu"], WORKLOAD["eps"], "fp64") as s:
        s.sync()
        t1 = time.perf_counter()
        s.step(WORKLOAD["tau"], steps)
        s.sync()
        t2 = time.perf_counter()
        s.fields()
        t3 = time.perf_counter()
    return {"value": nx * ny * nz * steps / (t3 - t0), "unit": "field-point-steps/s", "steps": steps,
            "dtype": "f64", "init_s": round(t1 - t0, 4), "steps_s": round(t2 - t1, 4),
            "fields_s": round(t3 - t2, 4)}


def summarize(prec: str, steps: int, wall: float, pass_ms: dict, inv: dict):
    nx, ny, nz = WORKLOAD["grid"]
    ns = nx * ny * nz
    tsize = 8 if prec == "fp64" else 4
    ms_per_step = 1e3 * wall / steps
    per_step = {k: v / steps for k, v in pass_ms.items()}
    # algorithmic bytes: every pass, the combined x kernel included, reads and writes the
    # state (6 components x N_S reals) once.  Per step of the K timed steps: z forward,
    # fused y and z inverse once; the x slots hold one x forward, K - 1 combined kernels
    # and one x inverse.
    state = 6.0 * ns * tsize
    slot_bytes = {"x_fwd": 2 * state / steps, "z_fwd": 2 * state, "y_fused": 2 * state, "z_inv": 2 * state,
                  "x_inv": 2 * state}
    # the dominant kernel: the longest launch.  The z, fused and x-inverse slots have one
    # launch per step (the x-inverse slot's are the combined kernel but for the last), so
    # their time and bytes per step are per launch.
    dominant = max(("z_fwd", "y_fused", "z_inv", "x_inv"), key=lambda k: per_step[k])
    avg_ms = per_step[dominant]
    alg_bytes = slot_bytes[dominant]
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(prec, KERNEL_NAMES[dominant])
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                "kernel": KERNEL_NAMES[dominant], "pass": dominant,
                "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": round(avg_ms, 5)}
    # the same launch against the vector-ALU issue ceiling (instructions per launch from
    # the committed SQ counters of the same kernel sources)
    valu = measured_valu(prec, KERNEL_NAMES[dominant])
    issue = None
    if valu is not None:
        gips = valu / (avg_ms * 1e-3) / 1e9
        issue = {"bound": "alu", "achieved": round(gips, 1), "peak": PEAK_VALU_GIPS,
                 "unit": "G VALU wave-instructions/s", "frac": round(gips / PEAK_VALU_GIPS, 4),
                 "kernel": KERNEL_NAMES[dominant], "valu_per_launch": valu}
    step_bytes = sum(slot_bytes.values())
    value = ns / (ms_per_step * 1e-3)
    # the step's HBM bytes as the counters count them (committed summary of the same
    # kernels): per call one x forward, K z forward + z inverse (the summary's k_c2c
    # figure averages the two), K fused passes, K - 1 combined x kernels, one x inverse
    counted = {k: measured_traffic(prec, k) for k in ("k_x_fwd", "k_c2c", "k_fused", "k_x_invfwd", "k_x_inv")}
    counted_gbs = None
    if all(v is not None for v in counted.values()):
        per_call = (counted["k_x_fwd"] + steps * (2 * counted["k_c2c"] + counted["k_fused"]) +
                    (steps - 1) * counted["k_x_invfwd"] + counted["k_x_inv"])
        counted_gbs = round(per_call / steps / (ms_per_step * 1e-3) / 1e9, 1)
    return {
        "value": value,
        "ms_per_step": ms_per_step,
        "pass_ms_per_step": {k: round(v, 5) for k, v in per_step.items()},
        "roofline": roofline,
        "issue": issue,
        "step_alg_bytes": step_bytes,
        "step_hbm_gbs": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1),
        # HBM traffic of the step by the counters, and its fraction of the 8 TB/s peak
        "step_counted_gbs": counted_gbs,
        "step_counted_frac": round(counted_gbs / PEAK_HBM_GBS, 4) if counted_gbs else None,
        # the method's irreducible traffic: read and write the six fields once per step
        "method_alg_frac": round(value * 12 * tsize / (PEAK_HBM_GBS * 1e9), 4),
        "energy": inv["energy"],
    }


def copy_ceiling(nbytes: int, reps: int = 5):
    """Attainable HBM bandwidth on this GPU: a plain device-to-device copy of nbytes
    (read + write counted), timed with events, best of reps."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    best = None
    for _ in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del x, y
    return {"bytes": nbytes, "gbs": round(2 * nbytes / (best * 1e-3) / 1e9, 1)}


def host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


_CPU_FIELDS = None  # the inputs, inherited by the forked oracle processes


def _oracle_step(_=None):
    from oracle import oracle as orc
    H, E = _CPU_FIELDS
    t0 = time.perf_counter()
    orc.step(H, E, WORKLOAD["domain"], WORKLOAD["mu"], WORKLOAD["eps"], WORKLOAD["tau"], 1)
    return time.perf_counter() - t0


def cpu_baseline(H, E):
    """The FP64 CPU oracle as it stands on the same 256^3 workload: one step on one thread,
    then one step in each of P concurrent single-threaded processes (P = the host's CPU
    count, at most 16; the oracle has no threads of its own), whose aggregate rate is the
    reported value.  Runs before anything touches the GPU, so the worker processes are
    forked from a process with no device state."""
    import multiprocessing as mp
    global _CPU_FIELDS
    _CPU_FIELDS = (H, E)
    pts = int(H[0].size)
    single = _oracle_step()
    print(f"[bench] cpu oracle, one thread: {single:.2f} s/step", file=sys.stderr, flush=True)
    procs = max(1, min(os.cpu_count() or 1, 16))
    with mp.get_context("fork").Pool(procs) as pool:
        t0 = time.perf_counter()
        each = pool.map(_oracle_step, range(procs), chunksize=1)
        wall = time.perf_counter() - t0
    _CPU_FIELDS = None
    return {"value": procs * pts / wall, "unit": "field-point-steps/s", "cores": procs, "kind": "oracle",
            "sample": f"1 step of the {round(pts ** (1 / 3))}^3 workload (full grid), FP64, in each of {procs} "
                      "concurrent single-threaded processes",
            "seconds": round(wall, 2), "max_process_s": round(max(each), 2),
            "single_thread": {"value": pts / single, "cores": 1, "seconds": round(single, 2)},
            "host": host_cpu()}


def serving(n_requests: int):
    from paper_2210_06232_amd import serving as sv

    def note(msg):
        print(f"[bench] serving {msg}", file=sys.stderr, flush=True)

    lat = sv.run_stream(n_requests, load=0.8, pool=1, modes=("batched", "serial_fp64"), progress=note)
    thr = sv.run_stream(n_requests, pool=1, modes=("batched", "serial_own", "serial_fp64", "anchored"), burst=True,
                        progress=note)

    def pick(r):
        keys = ("p50_s", "p99_s", "slowdown_p50", "slowdown_p99", "point_steps_per_s", "wall_s", "completed",
                "failed", "peak_running", "mean_batch", "peak_bytes")
        return {k: (round(r[k], 6) if isinstance(r[k], float) else r[k]) for k in keys}

    return {
        "stream": f"{n_requests} requests, grids 32^3..256^3 and 64x128x256, 70% fp32, nsteps log-uniform "
                  "[10,5000], cadence U{10..500}, budget 24 GB, max batch 32",
        "latency_load0.8": {"rate_per_s": round(lat["rate_per_s"], 4), "batched": pick(lat["batched"]),
                            "serial_fp64": pick(lat["serial_fp64"])},
        # serial solves in each request's own precision separate the batching gain from
        # the precision gain
        "throughput_burst": {"batched": pick(thr["batched"]), "serial_own": pick(thr["serial_own"]),
                             "serial_fp64": pick(thr["serial_fp64"]),
                             "speedup_vs_serial_fp64": round(thr["batched"]["point_steps_per_s"]
                                                             / thr["serial_fp64"]["point_steps_per_s"], 3),
                             "speedup_vs_serial_own": round(thr["batched"]["point_steps_per_s"]
                                                            / thr["serial_own"]["point_steps_per_s"], 3)},
        # outputs computed by jumps from each request's stored initial spectrum (the
        # scheme's exact flow over any span): same results up to rounding, steps between
        # outputs are not executed, so its point-steps/s is not comparable to stepping
        "anchored_burst": pick(thr["anchored"]),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=48, help="requests per serving replay (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(value is the one GPU's throughput)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    H, E = headline_inputs()
    print(f"[bench] inputs ready {H.shape}", file=sys.stderr, flush=True)
    cpu = None
    if rank == 0 and not args.no_cpu_baseline:
        cpu = cpu_baseline(H, E)
        print(f"[bench] cpu oracle, {cpu['cores']} processes: {cpu['value']:.3e} field-point-steps/s",
              file=sys.stderr, flush=True)
    r64, r32 = run_gpu_pair(H, E, args.steps, args.warmup)
    print(f"[bench] fp64 {r64['ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)
    print(f"[bench] fp32 {r32['ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)
    h2h = host_to_host(H, E, args.steps)
    print(f"[bench] fp64 host to host {h2h['value']:.3e} field-point-steps/s "
          f"(init {h2h['init_s']} s, fields {h2h['fields_s']} s)", file=sys.stderr, flush=True)
    nx, ny, nz = WORKLOAD["grid"]
    copy = copy_ceiling(6 * nx * ny * nz * 8)
    print(f"[bench] plain copy {copy['gbs']} GB/s", file=sys.stderr, flush=True)
    serve = None
    if args.serve_requests > 0:
        serve = serving(args.serve_requests)
        print(f"[bench] serving p50 {serve['latency_load0.8']['batched']['p50_s']:.3f} s", file=sys.stderr,
              flush=True)
    out = {
        "metric": "field-point-steps/s at 256^3 FP64 vs FP32 (% HBM roofline); served p50/p99 latency",
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
        # the dominant kernel against the vector-ALU issue ceiling (null while the SQ
        # counter summary was taken on other kernel sources)
        "issue": r64["issue"],
        "cpu_baseline": cpu,
        # attainable bandwidth (plain copy of the FP64 state) and the method's irreducible
        # traffic fraction (12 words per point-step) against the 8 TB/s peak
        "copy_ceiling": copy,
        "method_alg_frac": r64["method_alg_frac"],
        "step_hbm_gbs": r64["step_hbm_gbs"],
        "step_counted_gbs": r64["step_counted_gbs"],
        "step_counted_frac": r64["step_counted_frac"],
        "step_counted_note": "FETCH_SIZE/WRITE_SIZE count L2-to-fabric traffic, reads served by the 256 MB "
                             "last-level cache (MALL) included; gfx950 exposes no counter below the L2",
        "pass_ms_per_step": r64["pass_ms_per_step"],
        # the same K FP64 steps with the upload from and the download to host arrays
        "host_to_host": h2h,
        "fp32": {"value": r32["value"], "ms_per_step": r32["ms_per_step"], "dtype": "f32",
                 "roofline": r32["roofline"], "issue": r32["issue"], "pass_ms_per_step": r32["pass_ms_per_step"],
                 "method_alg_frac": r32["method_alg_frac"], "step_hbm_gbs": r32["step_hbm_gbs"],
                 "step_counted_gbs": r32["step_counted_gbs"], "step_counted_frac": r32["step_counted_frac"]},
        "serving": serve,
        "kernel_source_hash": kernel_source_hash(),
    }
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
