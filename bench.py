"""Benchmark of the EM-FEMPIC hot path on one MI355X.

Metric: particle-steps per second of the particle phase (sort + gather + push
+ track + deposit + deterministic reduction), timed with HIP events on the
library's stream; the full step (with the implicit field solve) is reported
beside it.  Workload: 40^3 Kuhn cube (384 000 tets), order-2 bases, 16M
electrons with a 1% sinusoidal density perturbation along x and a thermal
spread of 0.02 c, dt = 10 x the explicit-limit bound, PEC walls, mixed
precision; the plain FP64 path on the same workload is timed beside it.

Prints ONE JSON line.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_2111_12411_amd as F  # noqa: E402
from paper_2111_12411_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(order, precision, n_particles, n_tet):
    """Bytes the particle kernel must move per launch (one step):
    particle state read + write, plus per-tet field coefficients, DoF maps and
    geometry read once and the per-tet current partials written once."""
    rs = 4 if precision == F.MIXED else 8
    state = 6 * 8 + 18 * rs + 4  # r, v (FP64), 3 v-history, 3 a-history (rs), tet
    n1, n2 = (6, 4) if order == 1 else (20, 15)
    per_tet = 16 * 8 + (n1 + n2) * (rs + 4) + n1 * 8
    return 2 * state * n_particles + per_tet * n_tet, state, per_tet


def survey_bytes(order, precision, n_particles, n_tet, n1_int):
    """Algorithmic bytes of one particle phase (gather, push, track, deposit) in the model of the
    hot-path scope: particle state read and written once (r, v, the AB4 histories and the tet:
    196 B in FP64, 112 B in mixed precision with FP32 velocity and histories), per tet the field
    DoFs and geometry read once (516 B at order 2, 216 B at order 1) and the deposit partials
    written and read once (320 B, 96 B), and the deposit dg written once (8 B per interior W1 DoF).
    Sort traffic and spill records are not counted: they count against the implementation."""
    state = 196 if precision == F.FP64 else 112
    per_tet = (516 + 320) if order == 2 else (216 + 96)
    return 2 * state * n_particles + per_tet * n_tet + 8 * n1_int, state, per_tet


def boris_bytes(order, precision, n_particles, n_tet, n1_int):
    """The same model for the Boris push with a straight path: the state is the position,
    velocity (FP64) and tet, no histories (56 B in both precisions)."""
    _, _, per_tet = survey_bytes(order, precision, n_particles, n_tet, n1_int)
    state = 56
    return 2 * state * n_particles + per_tet * n_tet + 8 * n1_int, state, per_tet


def copy_bandwidth(gib=2, reps=5):
    """Measured device-to-device copy bandwidth (read + write bytes per second, GB/s) of a plain
    torch copy of `gib` GiB, the best of `reps` timed copies."""
    import torch
    n = (gib << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        t = a.elapsed_time(b) / 1e3
        best = t if best is None else min(best, t)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / best / 1e9


def pcg_bytes_per_iter(order, precision, rows, nnz, field_op=0, nt=0, inc=0):
    """Bytes one inner PCG iteration must move: q = A p with the fused dot(p, q); x, r and the
    preconditioned residual z updated with dot(r, z); p = z + beta p.  Inner vectors and values are
    FP32 in mixed precision, FP64 otherwise; order 2 has a 2x2 block-Jacobi preconditioner, order 1
    Jacobi.
    field_op 0: A assembled, at order 2 in 2x2 blocks with one int32 column per block, at order 1
    in CSR.  field_op 1: A applied tet by tet (nt tets): per tet its n1l local W1 ids (int32) and 16
    geometry words read, p read once, the n1l products written; then per row of A (int64 row
    pointers) its inc incidences (int32) and their products read, q written and p read again for
    the dot.  field_op 2 (order 2, DoF pairs): per tet one id and one product position (int32) per
    pair; the inc products of the rows written in row order and read contiguously, no incidences."""
    vs = 4 if precision == F.MIXED else 8
    if field_op:
        n1l = 20 if order == 2 else 6
        if field_op == 2:
            elem = nt * (n1l // 2) * 4 * 2 + nt * 16 * vs + rows * vs + inc * vs
            sums = (rows // 2 + 1) * 8 + inc * vs + 2 * rows * vs
        else:
            elem = nt * n1l * 4 + nt * 16 * vs + rows * vs + nt * n1l * vs
            sums = (rows + 1) * 8 + inc * 4 + inc * vs + 2 * rows * vs
        spmv = elem + sums
        precond = (rows // 2) * 4 * vs if order == 2 else rows * vs
    elif order == 2:
        blocks, brows = nnz // 4, rows // 2
        spmv = blocks * (4 * vs + 4) + brows * (8 + 3 * 2 * vs)  # values, column; row pointer, x, y, dot pairs
        precond = brows * 4 * vs
    else:
        spmv = nnz * (vs + 4) + rows * (8 + 3 * vs)
        precond = rows * vs
    update_xr = rows * 7 * vs + precond  # read x, p, r, q; write x, r, z
    update_p = rows * 3 * vs  # read z, p; write p
    return spmv + update_xr + update_p


def profiled_traffic():
    """HBM bytes per launch of k_particle<2, float> on the default workload, from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (copy-calibrated), or None
    when the kernel sources changed since those counters were taken."""
    try:
        txt = open(os.path.join(ROOT, "profiles", "k_particle_c3_mixed_hbm_counters.md")).read()
    except OSError:
        return None
    m1 = re.search(r"traffic_bytes_per_launch: (\S+)", txt)
    m2 = re.search(r"kernel_source_sha256: (\S+)", txt)
    if not (m1 and m2):
        return None
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h"):
        with open(os.path.join(ROOT, "paper_2111_12411_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return float(m1.group(1)) if h.hexdigest() == m2.group(1) else None


def run_workload(cfg_id, precision, steps, warmup, n=None, order=None, gauss_every=0, log=None, blocks=1,
                 pusher=F.PUSH_AB4):
    """Load the workload, take `warmup` steps, then time `steps` steps in `blocks` consecutive
    blocks; per block the device time of the particle phase and of its kernels (HIP events on the
    library's stream) comes from the run's statistics."""
    cfg = W.CONFIGS[cfg_id]
    N, k = cfg["N"], (cfg["order"] if order is None else order)
    mesh = F.Mesh.cube(N, k)
    info = mesh.info()
    dt = cfg["cfl"] * info["dt_cfl"]
    pos, vel = W.config_particles(cfg_id, n=n)
    npart = len(pos)
    w = W.config_weight(cfg_id, npart, dt)
    t0 = time.perf_counter()
    run = F.Run(mesh, dt, precision, pcg_rtol=1e-14, gauss_every=gauss_every, pusher=pusher)
    if log:
        run.set_log(log)
    run.load(pos, vel, -W.Q_E, W.M_E, w)
    t_setup = time.perf_counter() - t0
    del pos, vel
    run.step(warmup)
    run.sync()
    sizes = [steps // blocks + (1 if b < steps % blocks else 0) for b in range(blocks)]
    per_block = []
    t0 = time.perf_counter()
    for kb in sizes:
        run.step(kb)
        per_block.append((kb, run.stats()))
    run.sync()
    wall = time.perf_counter() - t0
    st = dict(per_block[-1][1])
    for key in ("particle_ms", "particle_kernel_ms", "continue_kernel_ms", "field_ms"):
        st[key] = sum(b[key] for _, b in per_block)
    t0 = time.perf_counter()
    rg = run.gauss()
    gauss_ms = (time.perf_counter() - t0) * 1e3
    e, b = run.fields()
    return dict(run=run, info=info, dt=dt, n=npart, wall=wall, stats=st, gauss=rg, gauss_ms=gauss_ms, setup_s=t_setup,
                e=e, b=b, blocks=per_block)


def rel(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


def oracle_threads():
    """Host threads of the oracle's all-cores leg: the CPUs this process may run on, at most 16
    (the host share of one GPU on the benchmark machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(cfg, n_sample, steps):
    """The FP64 oracle on a bounded sample of the workload: its plain C particle loop on all host
    threads (contiguous particle chunks, one deposit buffer per chunk, merged in chunk order) and,
    beside it, on one thread."""
    from oracle import core, mesh as omesh
    N, k = cfg["N"], cfg["order"]
    m = omesh.cube_mesh(N, k)
    # explicit-limit bound of the oracle at N=4, scaled by 4/N (similar meshes)
    m4 = omesh.cube_mesh(4, k)
    dt = cfg["cfl"] * core.cfl_dt(m4, core.assemble(m4)) * 4.0 / N
    threads = oracle_threads()
    legs = {}
    for name, nt_, n in (("all_cores", threads, n_sample * max(1, threads // 4)), ("one_thread", 1, n_sample)):
        pos, vel = W.config_particles(3, n=n)
        orc = core.OracleRun(m, dt, particles_only=True)
        orc.load(pos, vel, -W.Q_E, W.M_E, W.config_weight(3, n, dt))
        t0 = time.perf_counter()
        for _ in range(steps):
            orc.particle_step(threads=nt_)
        dtm = time.perf_counter() - t0
        legs[name] = (n * steps / dtm, n, dtm, nt_)
        del orc, pos, vel
    v, n, dtm, nt_ = legs["all_cores"]
    v1, n1, dtm1, _ = legs["one_thread"]
    return dict(value=v, unit="particle-steps/s", cores=nt_, kind="oracle",
                sample="%d particles x %d steps of the same workload (40^3 cube, order 2, zero fields), the "
                       "oracle's plain C loop on %d threads, %.1f s; one thread: %d particles x %d steps, %.1f s"
                       % (n, steps, nt_, dtm, n1, steps, dtm1),
                one_thread=dict(value=v1, unit="particle-steps/s", cores=1))


# plasma frequency times dt of the serving runs' macro weights: as for the largest run, the Debye
# length stays near a cell (at 0.1 the under-resolved plasma heats until paths cross more than
# 64 faces a step within the runs' 50-300 steps)
SERVING_OMEGA_DT = 0.01


def serving(n_jobs=64, slots=4, seed=4007, budget_gib=64):
    """The serving stream: n_jobs independent mixed-precision runs arrive with Poisson gaps and go
    through fempic_submit / fempic_poll.  Per run (numpy PCG64, seed 4007): N^3 cube with N uniform
    in [8, 30], order 1 or 2, 1e4-4e6 particles (log-uniform), beam (c2 shape) or thermal (v_th
    0.01c) at random, 50-300 steps, dt = 10 x the explicit bound.  The mean gap is half the mean
    time a run takes alone, measured first: four of the runs alone for 10 steps each, scaled by
    their step counts to the mean run.  Reports per-step latency (intervals between consecutive
    step completions of a run, over all runs: p50, p99), queue delay and aggregate
    particle-steps/s = sum n steps / makespan."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dt8 = {k: F.Mesh.cube(8, k).info()["dt_cfl"] for k in (1, 2)}  # Kuhn cubes: dt_cfl ~ 1/N
    specs = []
    for j in range(n_jobs):
        N = int(rng.integers(8, 31))
        k = int(rng.integers(1, 3))
        n = int(np.exp(rng.uniform(np.log(1e4), np.log(4e6))))
        kind = "beam" if rng.random() < 0.5 else "thermal"
        steps = int(rng.integers(50, 301))
        specs.append((N, k, n, kind, steps, 10.0 * dt8[k] * 8.0 / N))
    # mean isolated run time: four runs alone, 10 steps each, scaled to their step counts
    per_step = []
    for (N, k, n, kind, steps, dt) in specs[:4]:
        pos, vel = W.particles(kind, n, seed + 1000, vth=0.01, drift=0.1)
        run = F.Run(F.Mesh.cube(N, k), dt, F.MIXED, pcg_rtol=1e-13)
        run.load(pos, vel, -W.Q_E, W.M_E, W.plasma_weight(n, dt, omega_dt=SERVING_OMEGA_DT))
        run.step(2)
        run.sync()
        t0 = time.perf_counter()
        run.step(10)
        run.sync()
        per_step.append((time.perf_counter() - t0) / 10)
        run.close()
    mean_steps = float(np.mean([sp[4] for sp in specs]))
    iso_s = float(np.mean(per_step)) * mean_steps
    gaps = rng.exponential(0.5 * iso_s, n_jobs)
    jobs = []
    for j, (N, k, n, kind, steps, dt) in enumerate(specs):
        pos, vel = W.particles(kind, n, seed + j, vth=0.01, drift=0.1)
        jobs.append((N, k, pos, vel, W.plasma_weight(n, dt, omega_dt=SERVING_OMEGA_DT), steps, dt, n))
    srv = F.Server(hbm_budget=budget_gib << 30, max_slots=slots)
    t0 = time.perf_counter()
    tickets = []
    res = {}

    def drain():
        for t in tickets:
            if t not in res:
                r = srv.poll(t)
                if r is not None:
                    res[t] = r

    for j, (N, k, pos, vel, w, steps, dt, n) in enumerate(jobs):
        t_next = time.perf_counter() + gaps[j]
        while time.perf_counter() < t_next:
            drain()
            time.sleep(0.002)
        tickets.append(srv.submit(N, k, pos, vel, -W.Q_E, W.M_E, w, steps, dt, precision=F.MIXED))
    while len(res) < len(tickets):
        drain()
        time.sleep(0.002)
    makespan = time.perf_counter() - t0
    srv.close()
    lat, queue, failed, codes = [], [], 0, {}
    for t in tickets:
        r = res[t]
        if r["status"] != 0:
            failed += 1
            codes[str(r["status"])] = codes.get(str(r["status"]), 0) + 1
            continue
        lat.extend(np.diff(r["step_done_ms"]).tolist())
        queue.append(r["queue_ms"])
    work = sum(n * steps for (_, _, _, _, _, steps, _, n), t in zip(jobs, tickets) if res[t]["status"] == 0)
    return {"metric": "serving: per-step latency p50/p99 and aggregate particle-steps/s", "value": work / makespan,
            "unit": "particle-steps/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
            "p50_step_ms": float(np.percentile(lat, 50)), "p99_step_ms": float(np.percentile(lat, 99)),
            "queue_p50_ms": float(np.percentile(queue, 50)), "queue_max_ms": float(np.max(queue)),
            "makespan_s": makespan, "runs": n_jobs, "failed": failed, "failed_status": codes,
            "mean_gap_s": 0.5 * iso_s,
            "particle_steps": work,
            "config": {"workload": "%d runs, Poisson arrivals (mean gap %.2f s = half the mean isolated run time), "
                                   "%d slots, %d GiB budget; N in [8,30], order 1|2, 1e4-4e6 particles "
                                   "(log-uniform), beam|thermal, 50-300 steps, dt = 10 x explicit bound, "
                                   "omega_p dt = %g, mixed precision"
                                   % (n_jobs, 0.5 * iso_s, slots, budget_gib, SERVING_OMEGA_DT)}}


def beam_source(steps, warmup, n0=8_000_000, n_inj=40_000):
    """The beam experiment's shape on the benchmark mesh (40^3, order 2, mixed): a thermal
    plasma of n0 electrons, a beam of n_inj electrons injected through the wall z = 0 before
    every step (Table III's v0/c = 0.167), absorbing walls for particles and fields (the
    surface impedance matrix).  The rate counts the injection (host wall clock) with the
    particle phases."""
    import time
    cfg = W.CONFIGS[3]
    mesh = F.Mesh.cube(cfg["N"], cfg["order"])
    dt = 10.0 * mesh.info()["dt_cfl"]
    pos, vel = W.particles("thermal", n0, 3007, vth=0.02)
    w = W.plasma_weight(n0, dt, omega_dt=0.02)
    run = F.Run(mesh, dt, F.MIXED, pcg_rtol=1e-14, particle_bc=F.ABSORB, field_bc=F.FIELD_ABSORB)
    run.load(pos, vel, -W.Q_E, W.M_E, w)
    del pos, vel
    pstep = inj = 0.0
    ps = 0
    for k in range(warmup + steps):
        p, v = W.wall_beam(n_inj, 5000 + k)
        t0 = time.perf_counter()
        run.inject(p, v)
        t1 = time.perf_counter()
        run.step()
        st = run.stats()
        if k >= warmup:
            inj += t1 - t0
            pstep += st["particle_ms"] / 1e3
            ps += st["n_particles"] + st["absorbed"]  # the particles that moved in the step
    st = run.stats()
    g = run.gauss()
    run.close()
    return {"value": ps / (pstep + inj), "unit": "particle-steps/s", "steps": steps,
            "particle_ms_per_step": pstep * 1e3 / steps, "inject_ms_per_step": inj * 1e3 / steps,
            "injected_per_step": n_inj, "n_particles_end": st["n_particles"],
            "absorbed_total": st["absorbed_total"], "R_G": g[0], "R_C": g[1], "R_S": g[2],
            "config": "40^3 Kuhn cube, order 2, mixed; %d thermal electrons (v_th 0.02c) plus %d injected per step "
                      "at z = 0 (0.167c, radius 0.2); absorbing walls for particles and fields" % (n0, n_inj)}


def largest(steps, warmup, gauss_every=0, log=None):
    """The largest single-GPU run: 56^3 Kuhn cube (1 053 696 tets), order 2, 64M electrons in two
    counter-streaming beams at +-0.2c (thermal 0.01c), dt = 10 x explicit bound, mixed precision.
    gauss_every > 0 evaluates R_G, R_C, R_S every that many steps into the step log `log`."""
    r = run_workload(5, F.MIXED, steps, warmup, gauss_every=gauss_every, log=log)
    st = r["stats"]
    alg, _, _ = survey_bytes(2, F.MIXED, r["n"], r["info"]["n_tet"], r["info"]["n1_int"])
    pms, kms = st["particle_ms"], st["particle_kernel_ms"]
    out = {"metric": "particle-steps/sec (gather+push+deposit), largest single run", "value": r["n"] * steps / (pms / 1e3),
           "unit": "particle-steps/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": r["wall"] * 1e3 / steps, "particle_ms_per_step": pms / steps,
           "field_ms_per_step": st["field_ms"] / steps, "higher_is_better": True, "dtype": "f32+f64",
           "data": "synthetic",
           "config": {"workload": "56^3 Kuhn cube (1053696 tets), order 2, %d electrons in two streams at +-0.2c, "
                                  "v_th 0.01c, dt = 10 x explicit bound, PEC walls, mixed precision" % r["n"]},
           "gauss_residual": {"R_G": r["gauss"][0], "R_C": r["gauss"][1], "R_S": r["gauss"][2], "ms": r["gauss_ms"]},
           "crossings_per_particle_step": st["crossings"] / r["n"],
           "roofline": {"bound": "hbm", "kernel": "k_particle<2,float>", "kernel_ms": kms / steps,
                        "frac": alg / (kms / steps / 1e3) / 1e9 / HBM_PEAK_GBS,
                        "phase_frac": alg / (pms / steps / 1e3) / 1e9 / HBM_PEAK_GBS, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s"},
           "setup_s": r["setup_s"]}
    r["run"].close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--particles", type=int, default=None, help="override the particle count (testing)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true",
                    help="only the mixed order-2 run (no FP64 or order-1 comparison runs)")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000)
    ap.add_argument("--no-copy", action="store_true", help="skip the device copy-bandwidth measurement")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy (counter calibration for profiles)")
    ap.add_argument("--slots", type=int, default=4, help="resident runs in --serving mode")
    ap.add_argument("--largest", action="store_true",
                    help="the largest single run instead: 56^3 cube, order 2, 64M electrons in two streams, mixed")
    ap.add_argument("--gauss-every", type=int, default=0,
                    help="Gauss-law residuals every that many steps, into the --log step log")
    ap.add_argument("--log", default=None, help="append one JSON line per step of the measured run to this file")
    ap.add_argument("--serving", action="store_true",
                    help="measure the submit/poll server on a stream of independent runs instead")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1): the library runs one simulation per MI355X "
              "and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.serving:
        print(json.dumps(serving(slots=args.slots)))
        return
    if args.largest:
        print(json.dumps(largest(args.steps, args.warmup, args.gauss_every, args.log)))
        return
    cfg = W.CONFIGS[3]
    # torch before the library's first use, so both share one HIP runtime
    copy_gbs = copy_bandwidth() if not args.no_copy else None
    if args.calib_copy:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    mix = run_workload(3, F.MIXED, args.steps, args.warmup, n=args.particles, blocks=3, gauss_every=args.gauss_every,
                       log=args.log)
    st = mix["stats"]
    K = args.steps
    n, nt, n1i = mix["n"], mix["info"]["n_tet"], mix["info"]["n1_int"]
    # the particle phase's rate in each of three consecutive blocks of the timed steps; the
    # reported value is their median
    rates = [n * kb / (b["particle_ms"] / 1e3) for kb, b in mix["blocks"]]
    value = float(np.median(rates))
    pms = st["particle_ms"]
    kms = st["particle_kernel_ms"]
    kernel_s = kms / K / 1e3
    alg, state_b, tet_b = survey_bytes(cfg["order"], F.MIXED, n, nt, n1i)
    alg_build, state_build, tet_build = algorithmic_bytes(cfg["order"], F.MIXED, n, nt)
    achieved = alg / kernel_s / 1e9
    traffic = profiled_traffic() if args.particles is None else None
    it = max(st["pcg_iters"], 1)
    pcg_b = pcg_bytes_per_iter(cfg["order"], F.MIXED, st["a_rows"], st["a_nnz"], st["field_op"], nt, st["a_inc"])
    # the field phase per step divided by its inner iterations: it also holds the right-hand
    # side, the Faraday update and the FP64 refinement residuals, so the rate is a lower bound
    pcg_ms = st["field_ms"] / K / it
    out = {
        "metric": "particle-steps/sec (gather+push+deposit) at p=1/2, FP64 vs mixed; Gauss residual",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": mix["wall"] * 1e3 / K,
        "particle_ms_per_step": pms / K,
        "field_ms_per_step": st["field_ms"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "40^3 Kuhn cube (384000 tets), order 2, %d electrons, 1%% sinusoidal density "
                               "perturbation in x, v_th 0.02c, omega_p dt = 0.02, dt = 10 x explicit bound, PEC walls, "
                               "mixed precision" % n, "order": 2, "n_tet": nt,
                   "particles": n, "dt": mix["dt"], "omega_p_dt": W.CONFIGS[3]["omega_dt"]},
        "block_rates": rates,
        "gauss_residual": {"R_G": mix["gauss"][0], "R_C": mix["gauss"][1], "R_S": mix["gauss"][2],
                           "ms": mix["gauss_ms"]},
        "pcg": {"iters_last_step": st["pcg_iters"], "relres": st["pcg_relres"], "a_rows": st["a_rows"],
                "a_nnz": st["a_nnz"], "field_op": st["field_op"], "a_inc": st["a_inc"],
                "alg_bytes_per_iter": pcg_b, "ms_per_iter": pcg_ms,
                "gb_s": pcg_b / (pcg_ms / 1e3) / 1e9},
        "crossings_per_particle_step": st["crossings"] / n,
        "spills_per_particle_step": st["spills"] / n,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)",
                     "kernel": "k_particle<2,float>", "kernel_ms": kms / K,
                     "alg_bytes_per_launch": alg, "alg_bytes_per_particle_step": alg / n,
                     "state_bytes": state_b, "per_tet_bytes": tet_b,
                     # the same launch against the bytes this build's layout moves (FP64 velocity in
                     # mixed precision: 124-B state; 568 B per tet)
                     "build_model": {"alg_bytes_per_launch": alg_build, "state_bytes": state_build,
                                     "per_tet_bytes": tet_build,
                                     "frac": alg_build / kernel_s / 1e9 / HBM_PEAK_GBS},
                     "copy_gbs": copy_gbs, "frac_of_copy": (achieved / copy_gbs) if copy_gbs else None,
                     # the whole particle phase (a1-a6, all its kernels and host waits) against the
                     # same algorithmic bytes per step
                     "phase_frac": alg / (pms / K / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "phase_frac_of_copy": (alg / (pms / K / 1e3) / 1e9 / copy_gbs) if copy_gbs else None},
    }
    mix["run"].close()
    if not args.no_fp64:
        # the plain FP64 path on the same inputs and the same number of steps
        f64 = run_workload(3, F.FP64, K, args.warmup, n=args.particles)
        s2 = f64["stats"]
        k2 = K
        out["mixed_vs_fp64"] = {"steps": K + args.warmup, "e_rel": rel(mix["e"], f64["e"]),
                                "b_rel": rel(mix["b"], f64["b"])}
        alg2, _, _ = survey_bytes(cfg["order"], F.FP64, f64["n"], f64["info"]["n_tet"], f64["info"]["n1_int"])
        out["fp64"] = {"value": f64["n"] * k2 / (s2["particle_ms"] / 1e3), "unit": "particle-steps/s",
                       "particle_ms_per_step": s2["particle_ms"] / k2, "ms_per_step": f64["wall"] * 1e3 / k2,
                       "R_G": f64["gauss"][0],
                       "roofline_frac": alg2 / (s2["particle_kernel_ms"] / k2 / 1e3) / 1e9 / HBM_PEAK_GBS}
        f64["run"].close()
    if not args.no_fp64:
        # the same workload with order-1 bases, mixed and FP64
        out["order1"] = {}
        for name, prec in (("mixed", F.MIXED), ("fp64", F.FP64)):
            r1 = run_workload(3, prec, K, args.warmup, n=args.particles, order=1)
            s1 = r1["stats"]
            alg1, _, _ = survey_bytes(1, prec, r1["n"], r1["info"]["n_tet"], r1["info"]["n1_int"])
            out["order1"][name] = {"value": r1["n"] * K / (s1["particle_ms"] / 1e3), "unit": "particle-steps/s",
                                   "particle_ms_per_step": s1["particle_ms"] / K,
                                   "ms_per_step": r1["wall"] * 1e3 / K, "R_G": r1["gauss"][0],
                                   "crossings_per_particle_step": s1["crossings"] / r1["n"],
                                   "roofline_frac": alg1 / (s1["particle_kernel_ms"] / K / 1e3) / 1e9 / HBM_PEAK_GBS}
            r1["run"].close()
    if not args.no_fp64:
        # the alternative pusher on the same workload (mixed precision): throughput beside AB4
        rb = run_workload(3, F.MIXED, K, args.warmup, n=args.particles, pusher=F.PUSH_BORIS)
        sb = rb["stats"]
        algb, stb, _ = boris_bytes(cfg["order"], F.MIXED, rb["n"], rb["info"]["n_tet"], rb["info"]["n1_int"])
        out["boris"] = {"value": rb["n"] * K / (sb["particle_ms"] / 1e3), "unit": "particle-steps/s",
                        "particle_ms_per_step": sb["particle_ms"] / K, "kernel_ms": sb["particle_kernel_ms"] / K,
                        "ms_per_step": rb["wall"] * 1e3 / K, "R_G": rb["gauss"][0],
                        "crossings_per_particle_step": sb["crossings"] / rb["n"], "state_bytes": stb,
                        "roofline_frac": algb / (sb["particle_kernel_ms"] / K / 1e3) / 1e9 / HBM_PEAK_GBS}
        rb["run"].close()
        # injection and absorbing walls on the hot path
        out["beam_source"] = beam_source(K, args.warmup)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample, 2)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
