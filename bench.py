#!/usr/bin/env python
"""Benchmark of the serving cycle on the 16-human workload.

Workload: 16 humans with particle counts log-uniform in [2^14, 2^18]
(about 1.5e6 particles), 2-6 goals each, 9 beta values, 16 headings at
1.2 m/s, dt = 0.02 s, H = 100 steps, one 256x256 grid (0.05 m) per human.
One step = one serving cycle over all humans: a new observed position per
human, belief update, grid clear, one persistent batched rollout launch
(hipGraph), normalisation.  Synthetic data: humans are simulated on the GPU
by the library's Boltzmann-policy track simulator; all inputs are resident
before the timed region (only the per-cycle observation/descriptor copy,
about 16 x 3 KB, crosses PCIe, as it would in serving).

Reported: particle-steps/s of back-to-back batched cycles (`value`); the
same for the plain per-human sequential launches (the paper's multi-human
procedure, Sec. IV-B) and their ratio; p50/p99 latency of a 125 Hz paced
loop; the rollout kernel's roofline (live HIP-event timing); the 64-human
scene; the consumers (union of the grids, one MPPI step); the differentiable
log-likelihood and its adjoint on 1024 tracks; one Tab. 1-shaped prediction;
and the FP64 oracle timed on the host cores over whole cycles (at least 10 s).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9   # full-rate VALU lane operations per second (MI355X)
METRIC = "particle-steps/sec + p99 cycle latency, 16 humans @125Hz, batched vs plain"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_ops(K: int, r: dict) -> float:
    """Minimal VALU time per particle-step of the stable-form rollout, in
    full-rate lane-operation slots (one FP32 FMA = 1; rates r from the probes).
    Operation counts of the algorithm:
      per heading: dot product shared by the two opposite headings (1),
                   n_k = |s|^2 +- dot (1), |a|^2 + n_k (1), scaled
                   denominator FMA (1), exponent multiply (1), prefix add (1)
                   = 6 full-rate, plus sqrt, reciprocal and exp2;
      inverse CDF: binary search, log2(K) compare + select pairs;
      per step:    offset/convert/|a|^2/|a| scale/2a/uniform/threshold/step/
                   cell/bounds = 22 full-rate plus one sqrt;
      Philox:      one 10-round block per 4 steps = 5 wide multiplies and
                   10 full-rate ops per step.
    Transcendentals issue in one slot and then occupy their own pipe for
    r[kind] slots (the mixed probe -- one exp2 with four full-rate ops costs
    about five slots, not 3 + 4 -- shows the overlap), so the time is
    max(issue slots, transcendental pipe)."""
    issue, pipe = algorithmic_slots(K, r)
    return max(issue, pipe)


def algorithmic_slots(K: int, r: dict):
    """(issue slots, transcendental-pipe slots) per particle-step; see algorithmic_ops."""
    trans = K * 3 + 1
    issue = K * 6 + 2 * math.log2(K) + 22 + 10 + trans + 5 * r["mul64"]
    pipe = K * (r["sqrt"] + r["rcp"] + r["exp2"]) + r["sqrt"]
    return issue, pipe


def resource_use(rates, K, psteps, seconds, counters):
    """Each resource of the rollout against its peak over one launch: VALU
    issue and the transcendental pipe (algorithmic slots, see algorithmic_ops),
    LDS atomics (one add per particle-step into the step's window; the probe's
    scattered-address LDS atomic rate is the peak), device-scope global
    atomics (the profiled count per launch against the probe's rate) and HBM
    bytes (the profiled traffic against 8 TB/s).  counters: the profiled
    {"traffic", "global_atomics"} per launch, if current, else None."""
    issue, pipe = algorithmic_slots(K, rates)
    traffic = None if counters is None else counters["traffic"]
    atomics = None if counters is None else counters["global_atomics"]
    out = {"valu_issue": round(issue * psteps / seconds / PEAK_LANE_OPS, 4),
           "transcendental_pipe": round(pipe * psteps / seconds / PEAK_LANE_OPS, 4),
           "lds_atomic": round(psteps / seconds / rates["lds_atomic_lane_ops_per_s"], 4),
           "lds_atomic_peak_lane_ops_per_s": float(f"{rates['lds_atomic_lane_ops_per_s']:.4e}"),
           "global_atomic": None if atomics is None else
           round(atomics / seconds / rates["global_atomic_per_s"], 4),
           "global_atomics_per_launch": atomics,
           "global_atomic_peak_per_s": float(f"{rates['global_atomic_per_s']:.4e}"),
           "hbm": None if traffic is None else round(traffic / seconds / 8e12, 5)}
    return out


def measure_rates(capred, torch) -> dict:
    """Issue cost of each op kind relative to an FP32 FMA, from the probes."""
    cus = capred.device_cu_count()
    blocks = cus * 8
    sink = torch.zeros(blocks, dtype=torch.float32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    iters = 4096
    for kind in ("fma", "exp2", "sqrt", "rcp", "mul64", "mix", "lds_atomic"):
        capred.probe(kind, 64, blocks, sink)
        e0.record()
        capred.probe(kind, iters, blocks, sink)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        ops = blocks * 256 * 8 * iters
        out[kind] = ops / (ms * 1e-3)
    rates = {k: out["fma"] / v for k, v in out.items()}
    rates["fma_lane_ops_per_s"] = out["fma"]
    rates["lds_atomic_lane_ops_per_s"] = out["lds_atomic"]
    # device-scope atomic adds at scattered addresses over one 512x512 step
    # grid (1 MiB) and over a 1 GiB footprint; the faster is the peak
    iters = 64
    for log2w, name in ((18, "1MiB"), (28, "1GiB")):
        counts = torch.zeros(1 << log2w, dtype=torch.int32, device="cuda")
        capred.probe_global_atomic(4, blocks, counts)
        e0.record()
        capred.probe_global_atomic(iters, blocks, counts)
        e1.record()
        torch.cuda.synchronize()
        rates[f"global_atomic_{name}_per_s"] = blocks * 256 * 8 * iters / (e0.elapsed_time(e1) * 1e-3)
        total = int(counts.sum(dtype=torch.int64))
        assert total == blocks * 256 * 8 * (iters + 4), "global atomic probe lost adds"
        del counts
    rates["global_atomic_per_s"] = max(rates["global_atomic_1MiB_per_s"],
                                       rates["global_atomic_1GiB_per_s"])
    return rates


def simulate(capred, torch, np, humans, T):
    start = torch.tensor(np.array([h.start for h in humans]), dtype=torch.float64, device="cuda")
    beta = torch.tensor(np.array([h.true_beta for h in humans], np.float32), device="cuda")
    goal = torch.tensor(np.array([h.goals[h.true_goal] for h in humans], np.float32),
                        device="cuda")
    h0 = humans[0]
    _, pos = capred.simulate_tracks(h0.K, h0.speed, h0.dt, h0.frame, start, beta, goal, T,
                                    seed=0, stream_id=0)
    pos = pos.cpu().numpy()
    return {h.hid: pos[i] for i, h in enumerate(humans)}


def make_server(capred, humans, tuning, tracks):
    from paper_2603_01122_amd.serve import HumanRequest, Server
    h0 = humans[0]
    srv = Server(h0.K, h0.speed, h0.dt, len(humans), max(h.H for h in humans),
                 max(h.grid[3] for h in humans), max(h.grid[4] for h in humans),
                 max(h.G for h in humans), max(h.B for h in humans), tuning=tuning)
    for h in humans:
        srv.submit(HumanRequest(h.hid, capred.model_of(h), h.grid, h.N, h.H, tracks[h.hid][0]))
    return srv


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, max_seconds, n_cycles=10):
    """The FP64 oracle on whole serving cycles (belief update with the newest
    observation + Alg. 1 for all humans), on every host core this process may
    use: n_cycles whole cycles, or fewer if max_seconds run out first.  Its
    observations come from its own track simulator."""
    import numpy as np
    import oracle
    threads = oracle.default_threads()
    sims = {}
    for h in scene.humans:
        _, pos = oracle.simulate_tracks(K=h.K, speed=h.speed, dt=h.dt, frame=h.frame,
                                        start=np.array([h.start]), beta=[h.true_beta],
                                        goal=h.goals[h.true_goal][None], T=64, seed=0,
                                        stream=h.hid)
        sims[h.hid] = pos[0]
    lb = {h.hid: None for h in scene.humans}
    t0 = time.perf_counter()
    steps = 0
    cycles = 0
    humans_done = 0
    while cycles < 63:
        for h in scene.humans:
            obs = sims[h.hid][cycles:cycles + 2]
            lb[h.hid], b, _ = oracle.belief_update(K=h.K, speed=h.speed, dt=h.dt, beta=h.beta,
                                                   goals=h.goals, obs=obs, log_belief=lb[h.hid])
            oracle.predict(K=h.K, speed=h.speed, dt=h.dt, beta=h.beta, goals=h.goals, grid=h.grid,
                           z0=tuple(obs[-1].astype(float)), belief=b, N=h.N, H=h.H, seed=0,
                           human=h.hid, cycle=cycles, nthreads=threads)
            steps += h.N * h.H
            humans_done += 1
            if time.perf_counter() - t0 > max_seconds:
                break
        if time.perf_counter() - t0 > max_seconds:
            break
        cycles += 1
        if cycles >= n_cycles:
            break
    dt = time.perf_counter() - t0
    n_h = len(scene.humans)
    sample = (f"{cycles} full serving cycles of the {n_h}-human workload "
              f"({steps} particle-steps)" if humans_done == cycles * n_h else
              f"{humans_done} human-cycles of the {n_h}-human workload ({steps} particle-steps)")
    return {"value": steps / dt, "unit": "particle-steps/s", "cores": threads,
            "kind": "oracle", "sample": sample, "seconds": round(dt, 3),
            "cpu_model": cpu_model()}


def profiled_counters(best, scene="16humans"):
    """HBM bytes and device-scope atomics per rollout launch of a scene
    ("16humans" or "64humans") from the committed counter summary, if the
    rollout's sources and the scene's launch shape are those the counters were
    taken on; else None."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "plan_rollout_kernel_16humans_counters.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    pre = "" if scene == "16humans" else "scene64_"
    keys = ("source_sha256", "sources", pre + "tuning", pre + "traffic_bytes_per_launch",
            pre + "global_atomics_per_launch")
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.split(": ", 1)[0] in keys)
    if len(fields) != len(keys):
        return None
    h = hashlib.sha256()
    for src in fields["sources"].split():
        with open(os.path.join(here, src), "rb") as f:
            h.update(f.read())
    shape = "block_threads=%s particles_per_thread=%s" % (
        best.get("block_threads"), best.get("particles_per_thread"))
    for extra in ("lds_bytes", "grid_blocks"):
        if best.get(extra) is not None:
            shape += " %s=%s" % (extra, best[extra])
    if h.hexdigest() != fields["source_sha256"].strip() or shape != fields[pre + "tuning"].strip():
        return None
    return {"traffic": int(fields[pre + "traffic_bytes_per_launch"]),
            "global_atomics": int(fields[pre + "global_atomics_per_launch"])}


def mppi_timing(capred, torch, np, srv, humans, cycle, reps=20):
    """Union of the 16 humans' newest grids (point-wise max) and one MPPI step
    (N = 8192 samples, T = 40) of a robot crossing the scene, on the GPU right
    after a serving cycle: the prediction consumer of Sec. III-C."""
    probs = [srv.grids(h.hid, cycle)[1] for h in humans]
    grid = humans[0].grid
    T, N = 40, 8192
    r = np.random.default_rng(11)
    delta = torch.tensor(r.normal(scale=[0.8, 0.6], size=(T, N, 2)), device="cuda")
    U = torch.zeros((T, 2), dtype=torch.float64, device="cuda")
    S = torch.empty(N, dtype=torch.float64, device="cuda")
    occ = torch.empty_like(probs[0])
    z0, goal = (1.0, 1.0, 0.8, 0.7), (11.0, 11.0, 0.0, 0.0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tu, tm = [], []
    for k in range(reps + 2):
        ev[0].record()
        capred.union_max(probs, out=occ)
        ev[1].record()
        capred.mppi_step(z0, goal, U, delta, dt=humans[0].dt, tau=10.0, occ=occ, grid=grid, S=S,
                         **capred.PAPER_MPPI_COST)
        ev[2].record()
        torch.cuda.synchronize()
        if k >= 2:
            tu.append(ev[0].elapsed_time(ev[1]))
            tm.append(ev[1].elapsed_time(ev[2]))
    cells = occ.numel()
    return {"union_ms": round(float(np.median(tu)), 4),
            "union_GBps": round(cells * 4 * (len(probs) + 1) / (np.median(tu) * 1e-3) / 1e9, 1),
            "mppi_ms": round(float(np.median(tm)), 4), "samples": N, "horizon": T}


def loglik_timing(capred, torch, np, scenes, reps=20):
    """The differentiation workload: 1024 tracks of 200 transitions (K = 32,
    dt = 0.05 s, per-track beta and one of 8 goals, simulated on the GPU), the
    batched log-likelihood over 8 goals x 9 beta and its adjoint with respect
    to the goals and log beta (median of `reps` calls each)."""
    ts = scenes.config4()
    n = ts.starts.shape[0]
    start = torch.tensor(ts.starts, dtype=torch.float64, device="cuda")
    beta = torch.tensor(ts.true_beta, dtype=torch.float32, device="cuda")
    goal = torch.tensor(ts.goals[ts.true_goal], dtype=torch.float32, device="cuda")
    _, pos = capred.simulate_tracks(ts.K, ts.speed, ts.dt, ts.frame, start, beta, goal, ts.T,
                                    seed=0, stream_id=4)
    tracks = pos.contiguous()
    lengths = torch.full((n,), ts.T, dtype=torch.int32, device="cuda")
    goals = torch.tensor(ts.goals, device="cuda")
    log_beta = torch.tensor(np.log(ts.beta_grid).astype(np.float32), device="cuda")
    dLL = torch.ones((n, log_beta.numel(), goals.shape[0]), dtype=torch.float64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tf, tb = [], []
    for k in range(reps + 2):
        ev[0].record()
        capred.loglik(ts.K, ts.speed, ts.dt, tracks, lengths, goals, log_beta)
        ev[1].record()
        capred.loglik_backward(ts.K, ts.speed, ts.dt, tracks, lengths, goals, log_beta, dLL)
        ev[2].record()
        torch.cuda.synchronize()
        if k >= 2:
            tf.append(ev[0].elapsed_time(ev[1]))
            tb.append(ev[1].elapsed_time(ev[2]))
    terms = n * ts.T * goals.shape[0] * log_beta.numel()
    fwd, bwd = float(np.median(tf)), float(np.median(tb))
    # goal / per-track beta fit from perturbed goals (300 Adam steps)
    from paper_2603_01122_amd.fit import fit_goals_beta
    r = np.random.default_rng(1)
    goals0 = torch.tensor((ts.goals + r.normal(scale=0.4, size=ts.goals.shape)).astype(np.float32),
                          device="cuda")
    lb0 = torch.zeros((n, 1), dtype=torch.float32, device="cuda")
    fit_goals_beta(ts.K, ts.speed, ts.dt, tracks, lengths, goals0, lb0, iters=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = fit_goals_beta(ts.K, ts.speed, ts.dt, tracks, lengths, goals0, lb0, iters=300)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t0
    err = np.linalg.norm(res.goals.cpu().numpy().astype(np.float64) - ts.goals, axis=1)
    return {"tracks": n, "steps": ts.T, "goals": int(goals.shape[0]), "beta": int(log_beta.numel()),
            "K": ts.K, "forward_ms": round(fwd, 4), "backward_ms": round(bwd, 4),
            "policy_terms_per_s_forward": float(f"{terms / (fwd * 1e-3):.4e}"),
            "policy_terms_per_s_backward": float(f"{terms / (bwd * 1e-3):.4e}"),
            "fit": {"adam_steps": 300, "seconds": round(fit_s, 4),
                    "ms_per_step": round(fit_s / 300 * 1e3, 4),
                    "start_goal_error_m": 0.4,
                    "max_goal_error_m": round(float(err.max()), 5),
                    "objective_first_last": [round(res.objective[0], 5),
                                             round(res.objective[-1], 5)]}}


def largest_scene(capred, torch, np, tune, scenes, rates, cycles):
    """The 64-human x 2^20-particle, K = 32, H = 200 scene: batched cycles
    back to back and the rollout kernel's share of the ALU roofline."""
    sc = scenes.config5()
    humans = sc.humans
    tracks = simulate(capred, torch, np, humans, cycles + 4)
    shape = tune.shipped(humans) or {}
    srv = make_server(capred, humans, shape, tracks)
    try:
        srv.step({h.hid: tracks[h.hid][1] for h in humans})
        srv.drain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in range(1, 1 + cycles):
            srv.step({h.hid: tracks[h.hid][c + 1] for h in humans})
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / cycles
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)   # the library re-records both around the rollout launch
        e1.record(stream)
        durs = []
        for _ in range(3):
            srv.plan.replay_rollout(stream, e0, e1)
            torch.cuda.synchronize()
            durs.append(e0.elapsed_time(e1) * 1e-3)
        roll = float(np.mean(durs))
    finally:
        srv.close()
    # the per-human reference launches of the same scene (one warm cycle, then timed ones)
    plain_shape = tune.shipped(humans, plain=True) or {"block_threads": 512,
                                                       "particles_per_thread": 1}
    psrv = make_server(capred, humans, plain_shape, tracks)
    try:
        psrv.step({h.hid: tracks[h.hid][1] for h in humans}, plain=True)
        psrv.drain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in range(1, 1 + cycles):
            psrv.step({h.hid: tracks[h.hid][c + 1] for h in humans}, plain=True)
        torch.cuda.synchronize()
        plain_sec = (time.perf_counter() - t0) / cycles
    finally:
        psrv.close()
    psteps = sc.particle_steps
    W = algorithmic_ops(humans[0].K, rates)
    achieved = W * psteps / roll
    counters = profiled_counters(shape, "64humans")
    resources = resource_use(rates, humans[0].K, psteps, roll, counters)
    return {"workload": "64 humans x 2^20 particles, 6 goals, 9 beta, K=32, v=1.2 m/s, "
                        "dt=0.01 s, H=200, 512x512 grids at 0.02 m",
            "particle_steps_per_cycle": psteps, "cycles": cycles,
            "ms_per_cycle": round(sec * 1e3, 3), "value": float(f"{psteps / sec:.6e}"),
            "plain_ms_per_cycle": round(plain_sec * 1e3, 3),
            "batched_over_plain": round(plain_sec / sec, 3),
            "tuning": shape, "plain_tuning": plain_shape,
            "roofline": {"bound": "alu", "kernel": "plan_rollout_kernel",
                         "ms_per_launch": round(roll * 1e3, 3),
                         "ops_per_particle_step": round(W, 2),
                         "achieved": round(achieved / 1e12, 3),
                         "peak": round(PEAK_LANE_OPS / 1e12, 3), "unit": "Tlane-op/s",
                         "frac": round(achieved / PEAK_LANE_OPS, 4),
                         "traffic": None if counters is None else counters["traffic"],
                         "resources": resources}}


def churn_paced(capred, torch, np, scenes, tuning, n_cycles, rate):
    """Continuous batching under churn: the 125 Hz loop over a seeded schedule
    of arrivals and departures (scenes.config3_churn: 16 humans at first, then
    Poisson arrivals with stays of 200-1400 cycles, about 16-18 present).  The
    server has 16 slots and a particle budget equal to the 16-human workload's
    total N, so arrivals wait for a slot and for budget and join at cycle
    boundaries; arrivals and departures are handled after each release tick,
    inside that cycle's latency.  Every present human walks one simulated step
    per cycle (waiting ones too: they join from where they are)."""
    import dataclasses
    from paper_2603_01122_amd.serve import HumanRequest, Server, latency_summary, run_paced
    visits = scenes.config3_churn(n_cycles)
    T = max(v.depart - v.arrive for v in visits) + 2
    walkers = [dataclasses.replace(v.human, hid=v.hid) for v in visits]
    sims = simulate(capred, torch, np, walkers, T)
    budget = sum(h.N for h in scenes.config3().humans)
    h0 = walkers[0]
    srv = Server(h0.K, h0.speed, h0.dt, 16, 100, 256, 256, 6, 9, particle_budget=budget,
                 tuning=tuning)
    arrive, depart = {}, {}
    for v in visits:
        arrive.setdefault(v.arrive, []).append(v)
        depart.setdefault(v.depart, []).append(v)
    present = {}

    def before(c):
        for v in depart.get(c, []):
            srv.depart(v.hid)
            present.pop(v.hid, None)
        for v in arrive.get(c, []):
            srv.submit(HumanRequest(v.hid, capred.model_of(v.human), v.human.grid, v.human.N,
                                    v.human.H, sims[v.hid][0]))
            present[v.hid] = v
        for r in srv.waiting:
            r.last_xy = sims[r.hid][c - present[r.hid].arrive]

    def obs(c):
        return {hid: sims[hid][c - v.arrive + 1] for hid, v in present.items()}

    try:
        lat = run_paced(srv, obs, n_cycles, rate, before_step=before,
                        progress=(2000, lambda k: log(f"  churn {k} cycles")))
        recs = list(srv.records)[-n_cycles:]
    finally:
        srv.close()
    first = {}
    for r in recs:
        for hid in r.humans:
            first.setdefault(hid, r.cycle)
    waits = [first[v.hid] - v.arrive for v in visits if v.hid in first]
    out = latency_summary(lat, 1.0 / rate)
    out.update({"rate_hz": rate, "visits": len(visits), "admitted": len(first),
                "mean_humans": round(float(np.mean([len(r.humans) for r in recs])), 2),
                "mean_particle_steps_per_cycle": float(f"{np.mean([r.particle_steps for r in recs]):.4e}"),
                "max_wait_cycles": int(max(waits)), "mean_wait_cycles": round(float(np.mean(waits)), 2),
                "slots": 16, "particle_budget": budget})
    return out


def union_in_cycle(capred, torch, np, humans, tuning, tracks, cycles, start):
    """Back-to-back cycles of the 16-human workload with the union stage on
    (the point-wise maximum of the 16 humans' probabilities, which share one
    frame, written inside each cycle's graph), against the same cycles without it."""
    from paper_2603_01122_amd.serve import HumanRequest, Server
    h0 = humans[0]
    out = {}
    for name, union in (("without", None), ("with", (h0.grid, h0.H))):
        srv = Server(h0.K, h0.speed, h0.dt, len(humans), h0.H, 256, 256, 6, 9, tuning=tuning,
                     union=union)
        try:
            for h in humans:
                srv.submit(HumanRequest(h.hid, capred.model_of(h), h.grid, h.N, h.H,
                                        tracks[h.hid][start]))
            for c in range(start, start + 10):
                srv.step({h.hid: tracks[h.hid][c + 1] for h in humans})
            srv.drain()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for c in range(start + 10, start + 10 + cycles):
                srv.step({h.hid: tracks[h.hid][c + 1] for h in humans})
            torch.cuda.synchronize()
            out[name] = (time.perf_counter() - t0) / cycles
        finally:
            srv.close()
    return {"cycle_ms_without_union": round(out["without"] * 1e3, 4),
            "cycle_ms_with_union": round(out["with"] * 1e3, 4),
            "union_in_cycle_ms": round((out["with"] - out["without"]) * 1e3, 4),
            "cycles": cycles}


def tab1_latency(capred, torch, np, calls=50):
    """One prediction at the shape of the paper's Tab. 1 (1 human, n = 8192,
    50 x 50 grid at 0.1 m, 5 beta, 10 goals, 96 controls = 6 speeds x 16
    headings, dt = 0.5 s) for T = 2..10: belief update with the newest
    observation, rollout and normalisation, host to host (median of `calls`)."""
    r = np.random.default_rng(2026)
    speeds = np.array([0.25, 0.5, 0.75, 1.0, 1.25, 1.5])
    goals = r.uniform(0.0, 5.0, (10, 2)).astype(np.float32)
    beta = np.array([0.1, 0.5, 1.0, 5.0, 10.0], np.float32)
    m = capred.Model(16, 0.0, 0.5, beta, goals, speeds=speeds)
    grid = (0.0, 0.0, 0.1, 50, 50)
    _, pos = capred.simulate_tracks(16, 0.0, 0.5, grid[:3],
                                    torch.tensor([[2.5, 2.5]], dtype=torch.float64, device="cuda"),
                                    torch.tensor([2.0], dtype=torch.float32, device="cuda"),
                                    torch.tensor(goals[:1], device="cuda"), calls + 8,
                                    seed=1, speeds=speeds)
    obs = pos[0].contiguous()
    pos_h = pos[0].cpu().numpy().astype(np.float64)
    lb = capred.belief_reset(torch.empty((10, 5), dtype=torch.float64, device="cuda"))
    b = torch.empty_like(lb)
    out = {}
    for T in (2, 4, 6, 8, 10):
        counts = torch.empty((T, 50, 50), dtype=torch.int32, device="cuda")
        off = torch.empty(T, dtype=torch.int32, device="cuda")
        probs = torch.empty((T, 50, 50), dtype=torch.float32, device="cuda")
        times = []
        for i in range(calls + 3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            capred.belief_update(m, obs[i:i + 2], lb, b)
            capred.predict_occupancy(m, grid, (pos_h[i + 1, 0], pos_h[i + 1, 1]), b,
                                     8192, T, seed=0, cycle=i, counts=counts, offgrid=off)
            capred.normalize(counts, 8192, probs)
            torch.cuda.synchronize()
            if i >= 3:
                times.append(time.perf_counter() - t0)
        out[f"T{T}_ms"] = round(float(np.median(times)) * 1e3, 4)
    out["context"] = ("paper Tab. 1: 7-8 ms per prediction at T = 2..10 on an RTX 2080 Ti "
                      "(JAX/XLA with JIT); different hardware")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed batched cycles")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--plain-steps", type=int, default=30)
    ap.add_argument("--paced-cycles", type=int, default=10000)
    ap.add_argument("--rate", type=float, default=125.0)
    ap.add_argument("--churn-cycles", type=int, default=10000,
                    help="paced cycles under the arrival/departure schedule (0 skips them)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=40.0,
                    help="cap on the oracle's 10 whole cycles")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--retune", action="store_true",
                    help="autotune even where the package's table holds this device and workload")
    ap.add_argument("--tuning", type=str, default=None,
                    help="JSON launch shape for the batched rollout (skips its autotuning)")
    ap.add_argument("--plain-tuning", type=str, default=None,
                    help="JSON launch shape for the plain launches (skips their autotuning)")
    ap.add_argument("--no-tab1", action="store_true",
                    help="skip the Tab. 1-shaped single-prediction latencies")
    ap.add_argument("--largest-cycles", type=int, default=3,
                    help="timed cycles of the 64-human x 2^20 scene (0 skips it)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain copy of this many MiB (byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): the library has no "
              "multi-GPU path; humans would be sharded across GPUs with no exchange step.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2603_01122_amd import capred, scenes, tune
    from paper_2603_01122_amd.serve import run_paced

    scene = scenes.config3()
    humans = scene.humans
    psteps = scene.particle_steps
    n_tune = 2 * 9 * 10
    T = (args.warmup + args.steps + args.plain_steps + args.paced_cycles + n_tune + 64 +
         2 * (10 + args.steps))
    log(f"simulating {len(humans)} tracks x {T} steps")
    tracks = simulate(capred, torch, np, humans, T)

    rates = measure_rates(capred, torch)
    log(f"probe rates (cost relative to FMA): { {k: round(v, 3) for k, v in rates.items() if not k.endswith('_per_s')} }")

    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        capred.copy(a, b)
        torch.cuda.synchronize()
        log(f"copy calibration: {nbytes} bytes read and written by copy_kernel")
        del a, b
    best = json.loads(args.tuning) if args.tuning else ({} if args.no_tune else None)
    best_plain = (json.loads(args.plain_tuning) if args.plain_tuning
                  else ({} if args.no_tune else None))
    source = "flag"
    if best is None and not args.retune:
        best, source = tune.shipped(humans), "table"
    if best is None:
        best, _ = tune.autotune(humans, tracks, use_cache=False)
        source = "autotune"
    source_plain = "flag"
    if best_plain is None and not args.retune:
        best_plain, source_plain = tune.shipped(humans, plain=True), "table"
    if best_plain is None:
        best_plain, _ = tune.autotune(humans, tracks, plain=True, use_cache=False, cycles=3)
        source_plain = "autotune"
    log(f"launch shape batched: {best} ({source})  plain: {best_plain} ({source_plain})  "
        f"signatures {tune.signature(humans, False)} {tune.signature(humans, True)}")

    # ---------------------------------------------------------- batched, back-to-back
    srv = make_server(capred, humans, best, tracks)
    c = 0
    for _ in range(args.warmup):
        srv.step({h.hid: tracks[h.hid][c + 1] for h in humans})
        c += 1
    srv.drain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        srv.step({h.hid: tracks[h.hid][c + 1] for h in humans})
        c += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    srv.drain()
    sec_per_cycle = (t1 - t0) / args.steps
    value = psteps / sec_per_cycle
    log(f"batched: {1e3 * sec_per_cycle:.3f} ms/cycle, {value:.3e} particle-steps/s")

    # ---------------------------------------------------------- rollout kernel alone
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    e1.record(stream)
    durs = []
    for _ in range(20):
        srv.plan.replay_rollout(stream, e0, e1)
        torch.cuda.synchronize()
        durs.append(e0.elapsed_time(e1) * 1e-3)
    roll = float(np.mean(durs))
    W = algorithmic_ops(humans[0].K, rates)
    achieved = W * psteps / roll
    counters = profiled_counters(best)
    traffic = None if counters is None else counters["traffic"]
    roofline = {"bound": "alu", "achieved": round(achieved / 1e12, 3),
                "peak": round(PEAK_LANE_OPS / 1e12, 3), "unit": "Tlane-op/s",
                "frac": round(achieved / PEAK_LANE_OPS, 4), "traffic": traffic,
                # the same work per back-to-back cycle (consecutive rollouts overlap
                # their tails on the two streams): a serving-throughput view
                "cycle_frac": round(W * psteps / sec_per_cycle / PEAK_LANE_OPS, 4),
                "kernel": "plan_rollout_kernel", "ms_per_launch": round(roll * 1e3, 4),
                "ops_per_particle_step": round(W, 2),
                "particle_steps_per_launch": psteps,
                "rates_vs_fma": {k: round(v, 3) for k, v in rates.items()
                                 if not k.endswith("_per_s")},
                "fma_lane_ops_per_s": float(f"{rates['fma_lane_ops_per_s']:.4e}"),
                "global_atomic_per_s": {k: float(f"{rates[f'global_atomic_{k}_per_s']:.4e}")
                                        for k in ("1MiB", "1GiB")},
                "resources": resource_use(rates, humans[0].K, psteps, roll, counters)}
    log(f"rollout kernel {roll * 1e3:.3f} ms, {W:.1f} ops/particle-step, frac {achieved / PEAK_LANE_OPS:.3f}")

    # ---------------------------------------------------------- paced 125 Hz serving
    base = c
    lat = None
    if args.paced_cycles > 0:
        log(f"paced loop: {args.paced_cycles} cycles at {args.rate} Hz")
        lat = run_paced(srv, lambda k: {h.hid: tracks[h.hid][base + k + 1] for h in humans},
                        args.paced_cycles, args.rate,
                        progress=(2000, lambda k: log(f"  paced {k} cycles")))
        c += args.paced_cycles
    srv.drain()
    mppi = mppi_timing(capred, torch, np, srv, humans, c - 1)
    srv.close()
    mppi.update(union_in_cycle(capred, torch, np, humans, best, tracks, args.steps, c))
    log(f"union inside the cycle: {mppi['cycle_ms_with_union']} ms/cycle with, "
        f"{mppi['cycle_ms_without_union']} without")
    churn = None
    if args.churn_cycles > 0:
        log(f"paced loop under churn: {args.churn_cycles} cycles at {args.rate} Hz")
        churn = churn_paced(capred, torch, np, scenes, best, args.churn_cycles, args.rate)
        log(f"  churn: p50 {churn['p50_ms']} ms, p99 {churn['p99_ms']} ms, misses "
            f"{churn['deadline_misses']}, {churn['admitted']} of {churn['visits']} visits admitted")
    diff = loglik_timing(capred, torch, np, scenes)
    log(f"log-likelihood, 1024 tracks x 200 steps x 8 goals x 9 beta: forward "
        f"{diff['forward_ms']} ms, backward {diff['backward_ms']} ms")
    log(f"union of 16 grids {mppi['union_ms']} ms ({mppi['union_GBps']} GB/s), "
        f"MPPI step {mppi['mppi_ms']} ms")

    # ---------------------------------------------------------- plain per-human launches
    psrv = make_server(capred, humans, best_plain, tracks)
    for k in range(3):
        psrv.step({h.hid: tracks[h.hid][k + 1] for h in humans}, plain=True)
    psrv.drain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(3, 3 + args.plain_steps):
        psrv.step({h.hid: tracks[h.hid][k + 1] for h in humans}, plain=True)
    torch.cuda.synchronize()
    plain_sec = (time.perf_counter() - t0) / args.plain_steps
    psrv.close()
    plain_value = psteps / plain_sec
    log(f"plain: {1e3 * plain_sec:.3f} ms/cycle, {plain_value:.3e} particle-steps/s")

    largest = None
    if args.largest_cycles > 0:
        log("largest scene: 64 humans x 2^20 particles, K=32, H=200")
        largest = largest_scene(capred, torch, np, tune, scenes, rates, args.largest_cycles)
        log(f"  {largest['ms_per_cycle']} ms/cycle, {largest['value']:.3e} particle-steps/s, "
            f"rollout frac {largest['roofline']['frac']}, plain {largest['plain_ms_per_cycle']} "
            f"ms/cycle ({largest['batched_over_plain']}x)")

    tab1 = None
    if not args.no_tab1:
        log("Tab. 1-shaped latencies (n=8192, 50x50, 96 controls)")
        tab1 = tab1_latency(capred, torch, np)
        log(f"  {tab1}")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline (oracle, 10 whole cycles) on {cpu_model()}")
        cpu = cpu_baseline(scene, args.cpu_seconds)

    latency = None
    if lat is not None:
        from paper_2603_01122_amd.serve import latency_summary
        latency = latency_summary(lat, 1.0 / args.rate)
        latency["rate_hz"] = args.rate
        latency["mix"] = "static: the same 16 humans every cycle"
    if churn is not None:
        latency = latency or {}
        latency["churn"] = churn
    result = {
        "metric": METRIC,
        "value": float(f"{value:.6e}"),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec_per_cycle * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "16 humans, N log-uniform [2^14, 2^18] (sum %d), 2-6 goals, 9 beta, "
                               "K=16, v=1.2 m/s, dt=0.02 s, H=100, 256x256 grids at 0.05 m"
                               % sum(h.N for h in humans),
                   "particle_steps_per_cycle": psteps, "humans": len(humans),
                   "tuning": best, "plain_tuning": best_plain,
                   "tuning_source": [source, source_plain]},
        "latency": latency,
        "plain": {"value": float(f"{plain_value:.6e}"), "ms_per_step": round(plain_sec * 1e3, 4),
                  "batched_over_plain": round(value / plain_value, 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "largest_scene": largest,
        "consumer": mppi,
        "differentiation": diff,
        "tab1_shaped": tab1,
        "context": "paper: ~125 Hz for one human, n=8192, T=10, |U|=96 on an RTX 2080 Ti "
                   "(Tab. 1, JAX/XLA), about 1.0e7 particle-steps/s; different workload and hardware",
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
