"""GPU: the submit/poll server runs independent jobs concurrently, and each
job's result is bitwise the result of the same job run alone (the step is
deterministic and jobs share no state)."""
import time

import numpy as np
import pytest

import paper_2111_12411_amd as F
from paper_2111_12411_amd import workloads as W

pytestmark = pytest.mark.gpu

QE, ME = -W.Q_E, W.M_E


def _jobs():
    """(N, order, kind, n, seed, steps, precision): eight jobs over both orders, both precisions,
    beam and thermal particles and different mesh and particle sizes."""
    return [
        (4, 1, "thermal", 800, 11, 12, F.FP64),
        (6, 2, "beam", 3000, 12, 8, F.FP64),
        (5, 2, "thermal", 2000, 13, 10, F.MIXED),
        (4, 2, "beam", 1500, 14, 6, F.MIXED),
        (7, 1, "beam", 5000, 15, 9, F.MIXED),
        (3, 1, "thermal", 300, 16, 14, F.FP64),
        (8, 2, "thermal", 8000, 17, 5, F.FP64),
        (6, 1, "beam", 2500, 18, 11, F.MIXED),
    ]


def _alone(N, order, pos, vel, w, dt, steps, precision):
    run = F.Run(F.Mesh.cube(N, order), dt, precision, pcg_rtol=1e-13)
    run.load(pos, vel, QE, ME, w)
    run.step(steps)
    e, b = run.fields()
    p, v, _ = run.particles()
    rg = run.gauss()
    run.close()
    return e, b, p, v, rg


def test_server_matches_standalone_runs():
    specs = []
    for N, order, kind, n, seed, steps, prec in _jobs():
        dt = 5.0 * F.Mesh.cube(N, order).info()["dt_cfl"]
        pos, vel = W.particles(kind, n, seed, vth=0.01, drift=0.1)
        w = W.plasma_weight(n, dt)
        specs.append((N, order, pos, vel, w, dt, steps, prec))
    srv = F.Server(hbm_budget=8 << 30, max_slots=3)
    tickets = [srv.submit(N, order, pos, vel, QE, ME, w, steps, dt, precision=prec)
               for (N, order, pos, vel, w, dt, steps, prec) in specs]
    results = {}
    t0 = time.time()
    while len(results) < len(tickets):
        assert time.time() - t0 < 120, "server did not finish the jobs"
        for t in tickets:
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
        time.sleep(0.01)
    srv.close()
    for t, (N, order, pos, vel, w, dt, steps, prec) in zip(tickets, specs):
        r = results[t]
        assert r["status"] == 0, r["message"]
        e, b, p, v, rg = _alone(N, order, pos, vel, w, dt, steps, prec)
        assert np.array_equal(r["e"], e) and np.array_equal(r["b"], b)
        assert np.array_equal(r["pos"], p) and np.array_equal(r["vel"], v)
        assert len(r["step_done_ms"]) == steps and np.all(np.diff(r["step_done_ms"]) >= 0)
        if prec == F.FP64:
            assert r["gauss"][0] < 1e-12


def test_server_rejects_job_beyond_budget():
    srv = F.Server(hbm_budget=1 << 20, max_slots=1)  # 1 MiB: no run fits
    pos, vel = W.particles("thermal", 1000, 3)
    with pytest.raises(F.FempicError) as ex:
        srv.submit(8, 2, pos, vel, QE, ME, 1.0, 2, 1e-12)
    assert "ENOMEM" in str(ex.value)
    srv.close()


def test_server_isolates_a_failing_job():
    """A job with a NaN velocity fails with EINVAL at load; the jobs around it, one resident at a
    time, finish bitwise equal to the same jobs run alone."""
    specs = []
    for N, order, kind, n, seed, steps, prec in _jobs()[:2]:
        dt = 5.0 * F.Mesh.cube(N, order).info()["dt_cfl"]
        pos, vel = W.particles(kind, n, seed, vth=0.01, drift=0.1)
        specs.append((N, order, pos, vel, W.plasma_weight(n, dt), dt, steps, prec))
    bad = list(specs[0])
    bad_vel = bad[3].copy()
    bad_vel[7, 1] = np.nan
    bad[3] = bad_vel
    order = [specs[0], tuple(bad), specs[1]]
    srv = F.Server(hbm_budget=8 << 30, max_slots=1)
    tickets = [srv.submit(N, o, pos, vel, QE, ME, w, steps, dt, precision=prec)
               for (N, o, pos, vel, w, dt, steps, prec) in order]
    results = {}
    t0 = time.time()
    while len(results) < len(tickets):
        assert time.time() - t0 < 120, "server did not finish the jobs"
        for t in tickets:
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
        time.sleep(0.01)
    srv.close()
    assert results[tickets[1]]["status"] == -1 and "non-finite" in results[tickets[1]]["message"]
    for t, (N, o, pos, vel, w, dt, steps, prec) in ((tickets[0], specs[0]), (tickets[2], specs[1])):
        r = results[t]
        assert r["status"] == 0, r["message"]
        e, b, p, v, _ = _alone(N, o, pos, vel, w, dt, steps, prec)
        assert np.array_equal(r["e"], e) and np.array_equal(r["b"], b)
        assert np.array_equal(r["pos"], p) and np.array_equal(r["vel"], v)


def test_graph_replay_equals_eager_launches(monkeypatch):
    """The PCG batches replay a HIP graph captured once per run; with FEMPIC_GRAPHS=0 the same
    kernels launch one by one.  Every step (each replays the graph many times, with the run's
    own eager work and host reads between the replays) gives bit-identical fields, in both
    precisions and both orders."""
    for N, k, prec in ((5, 2, F.FP64), (5, 2, F.MIXED), (6, 1, F.MIXED)):
        dt = 10.0 * F.Mesh.cube(N, k).info()["dt_cfl"]
        pos, vel = W.particles("beam", 6000, 40 + N + k, vth=0.01, drift=0.1)
        w = W.plasma_weight(len(pos), dt)
        out = []
        for graphs in ("1", "0"):
            monkeypatch.setenv("FEMPIC_GRAPHS", graphs)
            run = F.Run(F.Mesh.cube(N, k), dt, prec, pcg_rtol=1e-14)
            run.load(pos, vel, QE, ME, w)
            steps = []
            for _ in range(6):
                run.step()
                steps.append(run.fields())
                assert run.stats()["pcg_iters"] >= 16
            out.append(steps)
            run.close()
        for (e1, b1), (e0, b0) in zip(*out):
            assert np.array_equal(e1, e0) and np.array_equal(b1, b0)


@pytest.mark.parametrize("N,k,prec,pusher,absorb", [
    (5, 2, F.MIXED, F.PUSH_AB4, False),
    (6, 1, F.FP64, F.PUSH_AB4, True),
    (5, 2, F.FP64, F.PUSH_BORIS, False),
])
def test_phase_graph_replay_equals_eager_launches(monkeypatch, N, k, prec, pusher, absorb):
    """With FEMPIC_PHASE_GRAPHS=1 the particle phase (k_particle to the next order) replays HIP
    graphs keyed by its launch bounds, captured when a key is new; the runs' own eager work (the
    field solve, host reads of the counts) lies between the replays.  Every one of 12 steps gives
    fields and particles bit-identical to eager launches, with walls reflecting or absorbing."""
    dt = 10.0 * F.Mesh.cube(N, k).info()["dt_cfl"]
    pos, vel = W.particles("beam", 6000, 70 + N + k, vth=0.02, drift=0.15)
    w = W.plasma_weight(len(pos), dt)
    out = []
    for graphs in ("1", "0"):
        monkeypatch.setenv("FEMPIC_PHASE_GRAPHS", graphs)
        kw = dict(pusher=pusher)
        if absorb:
            kw["particle_bc"] = F.ABSORB
        run = F.Run(F.Mesh.cube(N, k), dt, prec, pcg_rtol=1e-13, **kw)
        run.load(pos, vel, QE, ME, w)
        steps, replays = [], 0
        for _ in range(12):
            run.step()
            replays += run.stats()["phase_replays"]
            steps.append(run.fields() + run.particles()[:2])
        out.append(steps)
        run.close()
        # every step after the first (whose bounds are not known yet) replays a graph
        assert replays == (11 if graphs == "1" else 0)
    for a, b in zip(*out):
        for x, y in zip(a, b):
            assert np.array_equal(x, y, equal_nan=True)
