"""Serving on the GPU (through the C ABI): each solve gives the same bits alone, in a
mixed batch, with or without captured graphs, and through the plain solver; results
match the oracle within the FP64 / FP32 tolerances; snapshots hold the fields of the
step they report."""
import math
import time

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2210_06232_amd import inputs
from tests.helpers import elementwise_rel_error, energy_rel_error

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 2e-6
BUDGET = 8 << 30
CUBE = (0.0, 2 * math.pi, 0.0, 2 * math.pi, 0.0, 2 * math.pi)
BOX = (0.0, 2 * math.pi, 0.0, 4 * math.pi, 0.0, 8 * math.pi)


def eifp():
    from paper_2210_06232_amd import eifp as m
    m.load()
    return m


# (shape, domain, mu, eps, tau, nsteps, cadence, prec, workload seed)
A = ((32, 32, 32), CUBE, 1.0, 2.0, 0.05, 37, 10, "fp64", 11)
MIX = [
    A,
    ((32, 32, 32), CUBE, 1.0, 1.5, 0.08, 23, 5, "fp64", 12),
    ((32, 32, 32), CUBE, 1.0, 1.2, 0.02, 51, 0, "fp64", 13),
    ((32, 32, 32), CUBE, 1.0, 1.7, 0.05, 37, 10, "fp32", 14),
    ((16, 32, 64), BOX, 1.0, 1.1, 0.07, 29, 7, "fp64", 15),
    ((24, 24, 24), CUBE, 1.0, 1.9, 0.03, 44, 11, "fp32", 16),
    ((32, 32, 32), CUBE, 1.0, 1.3, 0.06, 19, 4, "fp32", 17),
]


def fields_of(case):
    shape, dom, *_, seed = case
    return inputs.random_fields(shape, dom, workload=seed, p=2.0)


def submit(sv, m, case, tag, flags=None):
    shape, dom, mu, eps, tau, nsteps, cad, prec, _ = case
    H, E = fields_of(case)
    fl = m.EIFP_REQ_KEEP_RESULT if flags is None else flags
    return sv.submit(H, E, dom, mu, eps, tau, nsteps, cad, prec, tag, fl)


def run(m, cases, max_batch=8, flags=0):
    """Submit every case, wait, return {tag: (H, E, step, [events])}."""
    out = {}
    with m.Server(BUDGET, max_batch, flags) as sv:
        ids = {submit(sv, m, c, i): i for i, c in enumerate(cases)}
        sv.drain(60000)
        evs = []
        while True:
            got = sv.poll(4096, 0)
            if not got:
                break
            evs += got
        st = sv.stats()
        assert st["failed"] == 0 and st["completed"] == len(cases), st
        for rid, i in ids.items():
            H, E, step = sv.fields(rid, cases[i][0])
            out[i] = (H, E, step, [e for e in evs if e["req_id"] == rid])
            sv.release(rid)
        assert sv.stats()["bytes_in_use"] >= 0
    return out, st


def solver_result(m, case):
    shape, dom, mu, eps, tau, nsteps, cad, prec, _ = case
    H, E = fields_of(case)
    with m.Solver(H, E, dom, mu, eps, prec) as s:
        s.step(tau, nsteps)
        Hs, Es = s.fields()
        inv = s.invariants()
    return Hs, Es, inv


def test_alone_equals_mix_equals_solver_bitwise():
    m = eifp()
    alone, _ = run(m, [A])
    mix, st = run(m, MIX)
    Ha, Ea, sa, eva = alone[0]
    Hm, Em, sm, evm = mix[0]
    assert sa == sm == A[5]
    assert np.array_equal(Ha, Hm) and np.array_equal(Ea, Em)
    # identical invariants at every output point
    assert [e["inv"] for e in eva] == [e["inv"] for e in evm]
    assert [e["step"] for e in eva] == [10, 20, 30, 37]
    # every member of the mix matches the plain solver bit for bit
    for i, case in enumerate(MIX):
        Hs, Es, inv = solver_result(m, case)
        Hg, Eg, step, evs = mix[i]
        assert step == case[5]
        assert np.array_equal(Hg, Hs) and np.array_equal(Eg, Es), i
        done = [e for e in evs if e["kind"] == "done"][0]
        assert done["inv"]["energy"] == inv["energy"] and done["inv"]["helicity"] == inv["helicity"], i
    assert st["chunks"] >= 1


def test_cancelled_member_leaves_its_batch_companions_unchanged():
    # an endless request shares a batch with A; cancelled after its first output, it ends
    # with one CANCELLED error event and no done event, and A still gives the plain
    # solver's bits
    m = eifp()
    endless = ((32, 32, 32), CUBE, 1.0, 1.4, 0.05, 10 ** 9, 20, "fp64", 21)
    with m.Server(BUDGET, 8) as sv:
        e_id = submit(sv, m, endless, 1, flags=0)
        a_id = submit(sv, m, A, 0)
        t0 = time.time()
        evs = []
        while not any(e["req_id"] == e_id and e["kind"] == "output" for e in evs):
            assert time.time() - t0 < 30, "no output from the endless request"
            evs += sv.poll(256, 100)
        sv.cancel(e_id)
        sv.drain(60000)
        while True:
            got = sv.poll(4096, 0)
            if not got:
                break
            evs += got
        st = sv.stats()
        mine = [e for e in evs if e["req_id"] == e_id]
        assert [e["kind"] for e in mine[:-1]] == ["output"] * (len(mine) - 1)
        assert mine[-1]["kind"] == "error" and mine[-1]["status"] == m.EIFP_ERR_CANCELLED
        assert st["cancelled"] == 1 and st["failed"] == 0 and st["completed"] == 1 and st["running"] == 0
        H, E, step = sv.fields(a_id, A[0])
        sv.release(a_id)
    Hs, Es, _ = solver_result(m, A)
    assert step == A[5] and np.array_equal(H, Hs) and np.array_equal(E, Es)


def test_mix_matches_oracle():
    m = eifp()
    mix, _ = run(m, MIX)
    for i, case in enumerate(MIX):
        shape, dom, mu, eps, tau, nsteps, cad, prec, _ = case
        H, E = fields_of(case)
        Ho, Eo, _ = orc.step(H, E, dom, mu, eps, tau, nsteps)
        Hg, Eg, _, _ = mix[i]
        # every FP32 rounding of a constant is compensated, so the FP32 error grows like the
        # square root of the step count and these runs (at most 51 steps) stay inside the
        # stated tolerance
        tol = FP64_TOL if prec == "fp64" else FP32_TOL
        en = energy_rel_error(Hg, Eg, Ho, Eo, mu, eps)
        el = elementwise_rel_error(Hg, Eg, Ho, Eo, mu, eps)
        print(f"case {i} {prec} {nsteps} steps: energy-norm {en:.3e}, element-wise {el:.3e}")
        assert en <= tol and el <= tol, (i, prec, en, el)


def test_graphs_and_eager_launches_agree_bitwise():
    m = eifp()
    g, _ = run(m, MIX)
    e, _ = run(m, MIX, flags=m.EIFP_SERVER_NO_GRAPHS)
    for i in g:
        assert np.array_equal(g[i][0], e[i][0]) and np.array_equal(g[i][1], e[i][1]), i


def test_small_batches_rotate_members():
    # six same-shape solves per precision through batches of two: a long first solve
    # keeps each batch busy while the short ones join and leave between chunks, so the
    # descriptors are repacked; every result still equals the solver's
    m = eifp()
    cases = [((24, 16, 32), CUBE, 1.0, 1.0 + 0.1 * j, 0.04 + 0.01 * j, (3000 if j < 2 else 13 + 6 * j), 3 + j,
              ("fp64", "fp32")[j % 2], 30 + j) for j in range(12)]
    res, st = run(m, cases, max_batch=2)
    assert st["peak_running"] >= 2
    for i, case in enumerate(cases):
        Hs, Es, _ = solver_result(m, case)
        assert np.array_equal(res[i][0], Hs) and np.array_equal(res[i][1], Es), i


def test_snapshot_is_the_reported_step():
    m = eifp()
    case = ((32, 32, 32), CUBE, 1.0, 2.0, 0.05, 4000, 25, "fp64", 21)
    shape, dom, mu, eps, tau, nsteps, cad, prec, _ = case
    H, E = fields_of(case)
    with m.Server(BUDGET, 4) as sv:
        rid = sv.submit(H, E, dom, mu, eps, tau, nsteps, cad, prec, 0, 0)
        # wait for the first output event, then read the latest snapshot
        t0 = time.time()
        evs = []
        while not evs and time.time() - t0 < 30:
            evs = sv.poll(16, 100)
        assert evs and evs[0]["kind"] == "output" and evs[0]["step"] == cad
        Hs, Es, step = sv.fields(rid, shape)
        assert step % cad == 0 and cad <= step < nsteps
        sv.drain(60000)
        with pytest.raises(m.EifpError):
            sv.fields(rid, shape)  # finished and not kept
    with m.Solver(H, E, dom, mu, eps, prec) as s:
        s.step(tau, step)
        Hr, Er = s.fields()
    assert np.array_equal(Hs, Hr) and np.array_equal(Es, Er)


def test_serial_mode_and_stats():
    m = eifp()
    res, st = run(m, MIX[:4], flags=m.EIFP_SERVER_SERIAL)
    assert st["peak_running"] == 1 and st["mean_batch"] == 1.0
    assert 0 < st["p50_s"] <= st["p99_s"] <= st["max_s"]
    assert st["point_steps"] == sum(np.prod(c[0]) * c[5] for c in MIX[:4])
    mix, _ = run(m, MIX[:4])
    for i in res:
        assert np.array_equal(res[i][0], mix[i][0]), i


def test_anchored_requests_match_solver_jumps_and_oracle():
    # anchored requests: every output is one jump from the stored initial spectrum; the
    # server's result equals the solver's eifp_jump bit for bit, and the oracle's single
    # step of nsteps * tau within tolerance (FP32 too, with no growth in nsteps)
    m = eifp()
    cases = [c[:5] + (c[5] * 20,) + c[6:] for c in MIX]  # 20x the steps: error must not grow
    res = {}
    with m.Server(BUDGET, 8) as sv:
        ids = {}
        for i, c in enumerate(cases):
            shape, dom, mu, eps, tau, nsteps, cad, prec, _ = c
            H, E = fields_of(c)
            ids[sv.submit(H, E, dom, mu, eps, tau, nsteps, cad, prec, i,
                          m.EIFP_REQ_KEEP_RESULT | m.EIFP_REQ_ANCHORED)] = i
        sv.drain(60000)
        evs = []
        while True:
            got = sv.poll(4096, 0)
            if not got:
                break
            evs += got
        st = sv.stats()
        assert st["failed"] == 0 and st["completed"] == len(cases)
        for rid, i in ids.items():
            res[i] = sv.fields(rid, cases[i][0])
            outs = [e["step"] for e in evs if e["req_id"] == rid]
            cad, n = cases[i][6], cases[i][5]
            assert outs == ([s for s in range(cad, n, cad)] if cad else []) + [n]
            sv.release(rid)
    for i, c in enumerate(cases):
        shape, dom, mu, eps, tau, nsteps, cad, prec, _ = c
        H, E = fields_of(c)
        with m.Solver(H, E, dom, mu, eps, prec) as s:
            s.jump(tau, nsteps)
            Hs, Es = s.fields()
        Hg, Eg, step = res[i]
        assert step == nsteps
        assert np.array_equal(Hg, Hs) and np.array_equal(Eg, Es), i
        Ho, Eo, _ = orc.step(H, E, dom, mu, eps, tau * nsteps, 1)
        tol = FP64_TOL if prec == "fp64" else FP32_TOL
        assert energy_rel_error(Hg, Eg, Ho, Eo, mu, eps) <= tol, (i, prec)


# States of 64 MiB or more get a work buffer, and their chunks run the x inverse of one
# step and the x forward of the next as one kernel (invariants on the chunk's last step
# only); the fields are still those of the plain solver, bit for bit, at every output.
BIG = [
    ((128, 128, 128), CUBE, 1.0, 1.4, 0.05, 9, 4, "fp64", 21),
    ((128, 128, 128), CUBE, 1.0, 1.8, 0.03, 6, 0, "fp64", 22),
    ((64, 128, 256), BOX, 1.0, 1.2, 0.04, 7, 3, "fp64", 23),
]


def test_large_states_step_with_the_combined_kernel_bitwise():
    m = eifp()
    assert m.eifp_server_footprint(128, 128, 128, "fp64") == 3 * 6 * 128 ** 3 * 8
    out, st = run(m, BIG)
    for i, case in enumerate(BIG):
        Hs, Es, inv = solver_result(m, case)
        Hg, Eg, step, evs = out[i]
        assert step == case[5]
        assert np.array_equal(Hg, Hs) and np.array_equal(Eg, Es), i
        done = [e for e in evs if e["kind"] == "done"][0]
        assert done["inv"]["energy"] == inv["energy"] and done["inv"]["helicity"] == inv["helicity"], i
        cad = case[6]
        want = [s for s in range(cad, case[5], cad)] if cad else []
        assert [e["step"] for e in evs if e["kind"] == "output"] == want, i
    assert st["completed"] == len(BIG)
