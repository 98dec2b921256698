"""Driver of the mixed-size serving stream: seeded Poisson arrivals of independent
EI-FP solves replayed in real time against the library's server, and the serial
baselines on the same arrivals.

Stream recipe (per request, seeded): grid uniform over STREAM_SHAPES; precision FP32
with probability 0.7, else FP64; nsteps log-uniform on [10, 5000]; output cadence
uniform on {10..500}; tau uniform on [0.01, 0.1]; mu = 1; eps uniform on [1, 2];
domain [0, 2 pi]^3, or [0, 2 pi] x [0, 4 pi] x [0, 8 pi] for the 64 x 128 x 256 grid
(the same spacing on every axis); initial fields from a pool of seeded random
divergence-free fields per shape.  The arrival rate is set from a calibrated service
time so that the offered load is a given fraction of one-at-a-time capacity in each
request's own precision.

Run: python -m paper_2210_06232_amd.serving --requests 2000 --load 0.8
"""
from __future__ import annotations

import argparse
import json
import math
import threading
import time

import numpy as np

from . import eifp, inputs

STREAM_SHAPES = [(32, 32, 32), (64, 64, 64), (96, 96, 96), (128, 128, 128), (192, 192, 192), (256, 256, 256),
                 (64, 128, 256)]
TWO_PI = 2.0 * math.pi
STREAM_SEED = 2210_06232 + 4000


def domain_of(shape):
    if shape == (64, 128, 256):
        return (0.0, TWO_PI, 0.0, 2 * TWO_PI, 0.0, 4 * TWO_PI)
    return (0.0, TWO_PI, 0.0, TWO_PI, 0.0, TWO_PI)


def make_stream(n_requests: int, seed: int = STREAM_SEED, pool: int = 1, max_steps: int = 5000):
    """Request parameters without arrival times (those depend on the rate)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_requests):
        shape = STREAM_SHAPES[int(rng.integers(len(STREAM_SHAPES)))]
        prec = "fp32" if rng.random() < 0.7 else "fp64"
        nsteps = int(round(math.exp(rng.uniform(math.log(10), math.log(max_steps)))))
        reqs.append(dict(tag=i, shape=shape, prec=prec, nsteps=nsteps, cadence=int(rng.integers(10, 501)),
                         tau=float(rng.uniform(0.01, 0.1)), mu=1.0, eps=float(rng.uniform(1.0, 2.0)),
                         domain=domain_of(shape), pool_index=int(rng.integers(pool))))
    return reqs


def add_arrivals(reqs, rate: float, seed: int = STREAM_SEED + 1):
    rng = np.random.default_rng(seed)
    t = 0.0
    for r in reqs:
        t += float(rng.exponential(1.0 / rate))
        r["arrival"] = t
    return reqs


def field_pools(reqs, pool: int, progress=None):
    """{(shape, index): (H, E)} for every pair the stream uses."""
    out = {}
    for r in reqs:
        key = (r["shape"], r["pool_index"])
        if key not in out:
            sid = 4000 + 10 * STREAM_SHAPES.index(r["shape"]) + r["pool_index"]
            out[key] = inputs.random_fields(r["shape"], r["domain"], workload=sid, p=2.0)
            if progress:
                progress(f"  fields {len(out)}: {key[0]} #{key[1]}")
    return out


def calibrate(pools, steps: int = 10):
    """Seconds per step of one solve on its own, per (shape, precision)."""
    out = {}
    for (shape, idx), (H, E) in pools.items():
        if idx:
            continue
        dom = domain_of(shape)
        for prec in ("fp32", "fp64"):
            with eifp.Solver(H, E, dom, 1.0, 1.5, prec) as s:
                s.step(0.05, 2)
                s.sync()
                t0 = time.perf_counter()
                s.step(0.05, steps)
                s.sync()
                out[(shape, prec)] = (time.perf_counter() - t0) / steps
    return out


def service_time(r, step_s, prec=None):
    return r["nsteps"] * step_s[(r["shape"], prec or r["prec"])]


def replay(reqs, pools, budget: int, max_batch: int = 32, flags: int = 0, force_prec=None, progress=None,
           step_s=None, req_flags: int = 0):
    """Submit each request at its arrival time (relative to the start) from a thread of
    its own, collect every event, and return the summary."""
    sv = eifp.Server(budget, max_batch, flags)
    done = {}
    n_out = [0]
    submit_lag = []
    errors = []

    def submitter():
        t0 = time.perf_counter()
        for r in reqs:
            dt = r["arrival"] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            H, E = pools[(r["shape"], r["pool_index"])]
            try:
                sv.submit(H, E, r["domain"], r["mu"], r["eps"], r["tau"], r["nsteps"], r["cadence"],
                          force_prec or r["prec"], r["tag"], req_flags)
            except Exception as ex:  # recorded, reported below
                errors.append((r["tag"], str(ex)))
            submit_lag.append(time.perf_counter() - t0 - r["arrival"])

    th = threading.Thread(target=submitter, daemon=True)
    wall0 = time.perf_counter()
    th.start()
    last_print = wall0
    while len(done) + len(errors) < len(reqs):
        for e in sv.poll(1024, 200):
            if e["kind"] == "output":
                n_out[0] += 1
            else:
                done[e["tag"]] = e
        now = time.perf_counter()
        if progress and now - last_print > 10:
            progress(f"  {len(done)}/{len(reqs)} done, {now - wall0:.0f} s")
            last_print = now
    th.join()
    wall = time.perf_counter() - wall0
    st = sv.stats()
    sv.close()
    failed = [t for t, e in done.items() if e["kind"] == "error"]
    pts = sum(float(np.prod(r["shape"])) * r["nsteps"] for r in reqs)
    extra = {}
    if step_s:
        # latency over the request's own service time alone (1 = no waiting, no sharing)
        slow = [(done[r["tag"]]["t_event"] - done[r["tag"]]["t_arrive"]) / service_time(r, step_s, force_prec)
                for r in reqs if r["tag"] in done]
        extra = {"slowdown_p50": float(np.percentile(slow, 50)), "slowdown_p99": float(np.percentile(slow, 99))}
    return {**extra, 
        "requests": len(reqs), "completed": st["completed"], "failed": len(failed) + len(errors),
        "outputs": n_out[0], "p50_s": st["p50_s"], "p99_s": st["p99_s"], "mean_s": st["mean_s"],
        "max_s": st["max_s"], "point_steps": pts, "wall_s": wall, "point_steps_per_s": pts / wall,
        "server_point_steps_per_s": st["point_steps_per_s"], "peak_running": st["peak_running"],
        "peak_bytes": st["peak_bytes"], "budget_bytes": budget, "chunks": st["chunks"],
        "mean_batch": st["mean_batch"], "submit_lag_p99_s": float(np.percentile(submit_lag, 99)),
    }


def run_stream(n_requests=64, load=0.8, pool=1, budget=24 * 10 ** 9, max_batch=32, modes=("batched", "serial_own",
               "serial_fp64"), max_steps=5000, progress=None, burst=False, rate=None):
    """Replay one seeded stream in each mode.  burst: every request arrives at t = 0
    (saturation: aggregate throughput); otherwise Poisson arrivals at `load` times the
    one-at-a-time capacity (latency), or at a given `rate` per second (then runs made
    separately, e.g. one mode per run, replay the same arrival times: the arrivals are
    seeded and depend only on the rate)."""
    reqs = make_stream(n_requests, pool=pool, max_steps=max_steps)
    pools = field_pools(reqs, pool, progress)
    step_s = calibrate(pools)
    mean_service = float(np.mean([service_time(r, step_s) for r in reqs]))
    if rate is None:
        rate = load / mean_service
    else:
        load = rate * mean_service  # the offered load this rate means on this GPU
    add_arrivals(reqs, rate)
    if burst:
        for r in reqs:
            r["arrival"] = 0.0
    out = {"requests": n_requests, "load": None if burst else round(load, 4), "burst": burst,
           "rate_per_s": None if burst else rate, "mean_service_s": mean_service, "pool": pool,
           "max_steps": max_steps, "budget_bytes": budget, "max_batch": max_batch,
           "step_ms": {f"{s[0]}x{s[1]}x{s[2]}_{p}": round(v * 1e3, 4) for (s, p), v in sorted(step_s.items())}}
    # mode: (max batch, server flags, forced precision, request flags)
    settings = {"batched": (max_batch, 0, None, 0),
                "batched_no_graphs": (max_batch, eifp.EIFP_SERVER_NO_GRAPHS, None, 0),
                "serial_own": (1, eifp.EIFP_SERVER_SERIAL, None, 0),
                "serial_fp64": (1, eifp.EIFP_SERVER_SERIAL, "fp64", 0),
                "anchored": (max_batch, 0, None, eifp.EIFP_REQ_ANCHORED)}
    for mode in modes:
        mb, fl, fp, rf = settings[mode]
        if progress:
            progress(f"{mode}: {n_requests} requests" + (" (burst)" if burst else f" at {rate:.2f}/s"))
        out[mode] = replay(reqs, pools, budget, mb, fl, fp, progress=progress, step_s=step_s, req_flags=rf)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--pool", type=int, default=8)
    ap.add_argument("--budget-gb", type=float, default=24.0)
    ap.add_argument("--max-batch", type=int, default=32)
    ap.add_argument("--max-steps", type=int, default=5000)
    ap.add_argument("--modes", default="batched,serial_own,serial_fp64",
                    help="comma list of batched, batched_no_graphs, serial_own, serial_fp64, anchored")
    ap.add_argument("--burst", action="store_true", help="every request arrives at t = 0")
    ap.add_argument("--rate", type=float, default=None,
                    help="arrivals per second (instead of --load), so that separate runs share one schedule")
    a = ap.parse_args()
    res = run_stream(a.requests, a.load, a.pool, int(a.budget_gb * 1e9), a.max_batch, tuple(a.modes.split(",")),
                     a.max_steps, progress=lambda s: print(s, flush=True), burst=a.burst, rate=a.rate)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
