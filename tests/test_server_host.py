"""Host logic of the serving loop, run without a GPU: the server's dry-run mode schedules
requests (admission by device footprint, batching by shape, chunking at output points,
events, statistics) exactly as the device mode does but allocates and launches nothing."""
import math
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2210_06232_amd", "libeifp.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libeifp.so not built")

CUBE = (0.0, 2 * math.pi, 0.0, 2 * math.pi, 0.0, 2 * math.pi)


def eifp():
    from paper_2210_06232_amd import eifp as m
    return m


def zeros(n):
    return np.zeros((3, n, n, n))


def events_by_request(evs):
    out = {}
    for e in evs:
        out.setdefault(e["req_id"], []).append(e)
    return out


def drain_events(sv):
    sv.drain(20000)
    evs = []
    while True:
        got = sv.poll(4096, 0)
        if not got:
            return evs
        evs += got


def test_footprint():
    m = eifp()
    assert m.eifp_server_footprint(32, 32, 32, "fp64") == 2 * 6 * 32 ** 3 * 8
    assert m.eifp_server_footprint(32, 32, 32, "fp32") == 2 * 6 * 32 ** 3 * 4
    assert m.eifp_server_footprint(32, 32, 32, "fp64", m.EIFP_REQ_NO_SNAPSHOT) == 6 * 32 ** 3 * 8
    assert m.eifp_server_footprint(64, 128, 256, "fp32") == 2 * 6 * 64 * 128 * 256 * 4
    # stepped requests with a state of 64 MiB or more add a work buffer (anchored ones
    # never step: none)
    s128 = 6 * 128 ** 3 * 8
    assert m.eifp_server_footprint(128, 128, 128, "fp64") == 3 * s128
    assert m.eifp_server_footprint(128, 128, 128, "fp64", m.EIFP_REQ_NO_SNAPSHOT) == 2 * s128
    assert m.eifp_server_footprint(128, 128, 128, "fp64", m.EIFP_REQ_ANCHORED) == 3 * s128
    assert m.eifp_server_footprint(128, 128, 128, "fp32") == 2 * s128 // 2
    assert m.eifp_server_footprint(256, 256, 256, "fp32") == 3 * 6 * 256 ** 3 * 4
    assert m.eifp_server_footprint(31, 32, 32, "fp64") == 0
    assert m.eifp_server_footprint(32, 32, 32, 7) == 0


def test_events_follow_the_cadence():
    m = eifp()
    with m.Server(1 << 30, 8, m.EIFP_SERVER_DRY_RUN) as sv:
        cases = [(8, 25, 10), (8, 30, 10), (16, 7, 0), (8, 1, 1), (16, 100, 7), (12, 5, 50)]
        ids = {}
        for tag, (n, nsteps, cad) in enumerate(cases):
            ids[sv.submit(zeros(n), zeros(n), CUBE, tau=0.1, nsteps=nsteps, cadence=cad, tag=tag)] = (tag, nsteps, cad)
        evs = events_by_request(drain_events(sv))
        assert set(evs) == set(ids)
        for rid, (tag, nsteps, cad) in ids.items():
            got = evs[rid]
            assert all(e["tag"] == tag for e in got)
            want = [s for s in range(cad, nsteps, cad)] if cad else []
            assert [e["step"] for e in got if e["kind"] == "output"] == want
            assert [e["kind"] for e in got][-1] == "done" and got[-1]["step"] == nsteps
            assert sum(e["kind"] == "done" for e in got) == 1
            assert all(e["status"] == 0 for e in got)
            assert all(abs(e["inv"]["t"] - 0.1 * e["step"]) < 1e-12 for e in got)
            assert all(e["t_arrive"] <= e["t_admit"] <= e["t_event"] for e in got)
        st = sv.stats()
        assert st["completed"] == len(cases) and st["failed"] == 0
        assert st["queued"] == 0 and st["running"] == 0
        assert st["point_steps"] == sum(n ** 3 * ns for n, ns, _ in cases)
        assert 0 <= st["p50_s"] <= st["p99_s"] <= st["max_s"]
        assert st["chunks"] >= 1 and st["mean_batch"] >= 1


def test_admission_respects_the_budget():
    m = eifp()
    fp = m.eifp_server_footprint(32, 32, 32, "fp64")
    # room for two requests plus the batch tables of one shape, not three requests
    budget = int(2.5 * fp)
    with m.Server(budget, 4, m.EIFP_SERVER_DRY_RUN) as sv:
        for i in range(12):
            sv.submit(zeros(32), zeros(32), CUBE, nsteps=2000, cadence=100, tag=i)
        evs = drain_events(sv)
        st = sv.stats()
    assert st["completed"] == 12
    assert st["peak_bytes"] <= budget
    assert st["peak_running"] <= 2
    assert sum(e["kind"] == "done" for e in evs) == 12


def test_serial_mode_runs_one_request_at_a_time():
    m = eifp()
    with m.Server(1 << 34, 16, m.EIFP_SERVER_DRY_RUN | m.EIFP_SERVER_SERIAL) as sv:
        for i in range(10):
            n = (8, 16, 32)[i % 3]
            sv.submit(zeros(n), zeros(n), CUBE, nsteps=50 + i, cadence=10, tag=i)
        evs = drain_events(sv)
        st = sv.stats()
    assert st["completed"] == 10 and st["peak_running"] == 1 and st["mean_batch"] == 1.0
    # one at a time, in arrival order
    done = [e["tag"] for e in evs if e["kind"] == "done"]
    assert done == list(range(10))


def test_submit_validation():
    m = eifp()
    z = zeros(8)
    bad = z.copy()
    bad[2, 1, 1, 1] = np.nan
    with m.Server(1 << 30, 4, m.EIFP_SERVER_DRY_RUN) as sv:
        cases = [
            (dict(H0=np.zeros((3, 8, 8, 7)), E0=np.zeros((3, 8, 8, 7))), m.EIFP_ERR_INVALID_ARG),
            (dict(H0=np.zeros((3, 8, 8, 10)), E0=np.zeros((3, 8, 8, 10))), m.EIFP_ERR_UNSUPPORTED_SIZE),
            (dict(nsteps=0), m.EIFP_ERR_INVALID_ARG),
            (dict(cadence=-1), m.EIFP_ERR_INVALID_ARG),
            (dict(tau=float("inf")), m.EIFP_ERR_INVALID_ARG),
            (dict(mu=0.0), m.EIFP_ERR_INVALID_ARG),
            (dict(domain=(0, 1, 1, 1, 0, 1)), m.EIFP_ERR_INVALID_ARG),
            (dict(H0=bad), m.EIFP_ERR_NONFINITE),
            (dict(prec=5), m.EIFP_ERR_INVALID_ARG),
        ]
        for kw, want in cases:
            args = dict(H0=z, E0=z, domain=CUBE, nsteps=10, cadence=0)
            args.update(kw)
            with pytest.raises(m.EifpError) as ei:
                sv.submit(**args)
            assert ei.value.status == want, kw
        with pytest.raises(m.EifpError) as ei:
            sv.fields(12345, (8, 8, 8))
        assert ei.value.status == m.EIFP_ERR_INVALID_ARG
        assert sv.stats()["submitted"] == 0
    # a footprint above the whole budget is refused at submit
    with m.Server(1000, 4, m.EIFP_SERVER_DRY_RUN) as sv:
        with pytest.raises(m.EifpError) as ei:
            sv.submit(z, z, CUBE, nsteps=10)
        assert ei.value.status == m.EIFP_ERR_OUT_OF_MEMORY


def test_create_validation_and_poll_without_work():
    m = eifp()
    with pytest.raises(m.EifpError):
        m.Server(0, 4, m.EIFP_SERVER_DRY_RUN)
    with pytest.raises(m.EifpError):
        m.Server(1 << 20, 0, m.EIFP_SERVER_DRY_RUN)
    with m.Server(1 << 20, 4, m.EIFP_SERVER_DRY_RUN) as sv:
        assert sv.poll(16, 0) == []
        assert sv.poll(16, -1) == []  # nothing queued or running: returns at once
        sv.drain(1000)


def test_kept_results_hold_memory_until_released():
    m = eifp()
    fp = m.eifp_server_footprint(16, 16, 16, "fp32")
    with m.Server(1 << 30, 4, m.EIFP_SERVER_DRY_RUN) as sv:
        rid = sv.submit(zeros(16), zeros(16), CUBE, nsteps=20, cadence=5, prec="fp32", flags=m.EIFP_REQ_KEEP_RESULT)
        drain_events(sv)
        # the snapshot half of the footprint is returned at completion; the state stays
        held = sv.stats()["bytes_in_use"]
        assert held >= fp // 2
        with pytest.raises(m.EifpError) as ei:
            sv.fields(rid, (16, 16, 16))  # dry run holds no data
        assert ei.value.status == m.EIFP_ERR_STATE
        sv.release(rid)
        assert sv.stats()["bytes_in_use"] == held - fp // 2
        with pytest.raises(m.EifpError):
            sv.release(rid)


def test_mixed_stream_batches_same_shapes():
    m = eifp()
    rng = np.random.default_rng(3)
    with m.Server(1 << 36, 32, m.EIFP_SERVER_DRY_RUN) as sv:
        shapes = [8, 12, 16]
        n_req = 60
        for i in range(n_req):
            n = shapes[rng.integers(3)]
            sv.submit(zeros(n), zeros(n), CUBE, nsteps=int(rng.integers(10, 3000)), cadence=int(rng.integers(10, 500)),
                      prec=("fp32", "fp64")[i % 2], tag=i)
        evs = drain_events(sv)
        st = sv.stats()
    assert st["completed"] == n_req and st["failed"] == 0
    assert sum(e["kind"] == "done" for e in evs) == n_req
    assert st["bytes_in_use"] >= 0


def test_anchored_requests_in_dry_run():
    m = eifp()
    fp = m.eifp_server_footprint(16, 16, 16, "fp64", m.EIFP_REQ_ANCHORED)
    assert fp == 3 * 6 * 16 ** 3 * 8
    with m.Server(1 << 30, 4, m.EIFP_SERVER_DRY_RUN) as sv:
        a = sv.submit(zeros(16), zeros(16), CUBE, nsteps=1000, cadence=250, flags=m.EIFP_REQ_ANCHORED, tag=1)
        b = sv.submit(zeros(16), zeros(16), CUBE, nsteps=1000, cadence=250, tag=2)
        evs = events_by_request(drain_events(sv))
        st = sv.stats()
    assert [e["step"] for e in evs[a]] == [250, 500, 750, 1000]
    assert [e["step"] for e in evs[b]] == [250, 500, 750, 1000]
    assert st["completed"] == 2


def test_injected_fault_fails_one_batch_and_the_server_goes_on(monkeypatch):
    # EIFP_SERVER_FAULT_CHUNK makes one chunk fail like a device error (host side, no GPU
    # involved): exactly the members of that batch end with an error event, their memory
    # goes back to the budget, and the rest of the stream completes
    m = eifp()
    monkeypatch.setenv("EIFP_SERVER_FAULT_CHUNK", "3")
    with m.Server(1 << 34, 4, m.EIFP_SERVER_DRY_RUN) as sv:
        ids = {}
        for i in range(6):
            n = (8, 16)[i % 2]
            ids[sv.submit(zeros(n), zeros(n), CUBE, nsteps=40, cadence=10, tag=i)] = i
        evs = events_by_request(drain_events(sv))
        st = sv.stats()
        errors = {rid for rid, es in evs.items() if any(e["kind"] == "error" for e in es)}
        done = {rid for rid, es in evs.items() if any(e["kind"] == "done" for e in es)}
        assert errors and not (errors & done) and errors | done == set(ids)
        for rid in errors:
            err = [e for e in evs[rid] if e["kind"] == "error"]
            assert len(err) == 1 and err[0]["status"] == m.EIFP_ERR_DEVICE
        assert st["failed"] == len(errors) and st["completed"] == len(done)
        assert st["running"] == 0 and st["queued"] == 0
        # the server still serves new requests after the fault
        later = sv.submit(zeros(8), zeros(8), CUBE, nsteps=5, cadence=0, tag=99)
        evs2 = events_by_request(drain_events(sv))
        assert [e["kind"] for e in evs2[later]] == ["done"]


def wait_for(sv, pred, timeout_s=10.0):
    import time
    t = time.time()
    while time.time() - t < timeout_s:
        st = sv.stats()
        if pred(st):
            return st
        time.sleep(0.002)
    raise AssertionError(f"server did not reach the state: {sv.stats()}")


def test_cancel_queued_and_running_requests():
    # two endless requests fill the budget, a third queues behind them; cancelling ends
    # the queued one at once and the running ones at a chunk boundary, each with one
    # CANCELLED error event, returns their memory, and later requests still run
    m = eifp()
    fp = m.eifp_server_footprint(32, 32, 32, "fp64")
    with m.Server(int(2.5 * fp), 4, m.EIFP_SERVER_DRY_RUN) as sv:
        a = sv.submit(zeros(32), zeros(32), CUBE, nsteps=10 ** 12, cadence=0, tag=1)
        b = sv.submit(zeros(32), zeros(32), CUBE, nsteps=10 ** 12, cadence=0, tag=2)
        wait_for(sv, lambda st: st["running"] == 2)
        c = sv.submit(zeros(32), zeros(32), CUBE, nsteps=5, cadence=0, tag=3)
        wait_for(sv, lambda st: st["queued"] == 1)
        sv.cancel(c)
        # again: a no-op while its event is pending; once the scheduler has ended it
        # (which may already have happened), the id is unknown
        try:
            sv.cancel(c)
        except m.EifpError as e:
            assert e.status == m.EIFP_ERR_INVALID_ARG
        sv.cancel(a)
        wait_for(sv, lambda st: st["cancelled"] == 2 and st["running"] == 1 and st["queued"] == 0)
        d = sv.submit(zeros(32), zeros(32), CUBE, nsteps=5, cadence=0, tag=4)
        wait_for(sv, lambda st: st["completed"] == 1)
        sv.cancel(b)
        evs = events_by_request(drain_events(sv))
        st = sv.stats()
        for rid in (a, b, c):
            assert [e["kind"] for e in evs[rid]] == ["error"], evs[rid]
            assert evs[rid][0]["status"] == m.EIFP_ERR_CANCELLED
        assert evs[c][0]["step"] == 0 and evs[a][0]["step"] > 0
        assert [e["kind"] for e in evs[d]] == ["done"]
        assert st["cancelled"] == 3 and st["completed"] == 1 and st["failed"] == 0
        assert st["running"] == 0 and st["queued"] == 0 and st["peak_bytes"] <= int(2.5 * fp)
        # ended requests are unknown to cancel; a kept result is released, not cancelled
        with pytest.raises(m.EifpError) as ei:
            sv.cancel(a)
        assert ei.value.status == m.EIFP_ERR_INVALID_ARG
        k = sv.submit(zeros(8), zeros(8), CUBE, nsteps=3, cadence=0, tag=5, flags=m.EIFP_REQ_KEEP_RESULT)
        drain_events(sv)
        with pytest.raises(m.EifpError) as ei:
            sv.cancel(k)
        assert ei.value.status == m.EIFP_ERR_STATE
        sv.release(k)


def test_cancel_under_load_keeps_the_accounting():
    # a stream of mixed requests with every third one cancelled at some point of its life
    # (queued, running or already ended): every request ends exactly once, as done or
    # cancelled, and all request memory returns to the budget
    import random
    m = eifp()
    rng = random.Random(5)
    fp = m.eifp_server_footprint(16, 16, 16, "fp64")
    with m.Server(int(6.5 * fp), 3, m.EIFP_SERVER_DRY_RUN) as sv:
        ids = []
        for i in range(60):
            n = (8, 16)[i % 2]
            ids.append(sv.submit(zeros(n), zeros(n), CUBE, nsteps=rng.choice((5, 200, 10 ** 6)),
                                 cadence=rng.choice((0, 50)), tag=i, prec=("fp64", "fp32")[i % 3 == 0]))
        asked = set()
        for rid in ids[::3]:
            try:
                sv.cancel(rid)
                asked.add(rid)
            except m.EifpError as e:  # already ended
                assert e.status == m.EIFP_ERR_INVALID_ARG
        # then cancel whatever is still live (the endless ones among them) so the stream ends
        evs = []
        for _ in range(200):
            evs += sv.poll(4096, 10)
            ended = {e["req_id"] for e in evs if e["kind"] in ("done", "error")}
            live = [r for r in ids if r not in ended]
            for rid in live:
                try:
                    sv.cancel(rid)
                    asked.add(rid)
                except m.EifpError:
                    pass
            if not live:
                break
        evs += drain_events(sv)
        st = sv.stats()
    by = events_by_request(evs)
    assert sorted(by) == sorted(ids)
    for rid, es in by.items():
        ends = [e for e in es if e["kind"] in ("done", "error")]
        assert len(ends) == 1 and es[-1] is ends[0], rid
        if ends[0]["kind"] == "error":
            assert ends[0]["status"] == m.EIFP_ERR_CANCELLED and rid in asked
    assert st["completed"] + st["cancelled"] == 60 and st["failed"] == 0
    assert st["running"] == 0 and st["queued"] == 0
    # what stays in use is the batch tables of idle groups, less than one request
    assert st["bytes_in_use"] < fp and st["peak_bytes"] <= int(6.5 * fp)
