"""GPU parity of the multi-speed control set (speeds x headings, the 96-control
experiments of Sec. IV) and of the speed mask of stationary humans (Sec. IV-B)
against the oracle, under the same bars as the one-speed path:

* simulated tracks: identical lattice positions;
* belief update (nearest-control recovery, U-control policy): the posterior's
  relative error 1e-5, i.e. |log b_gpu - log b_oracle| <= 1e-5 for every pair;
* prediction: first differences only at control-CDF ties within 1e-6, per-step
  histogram differences within 2 per flagged particle, TV <= 1e-3; masked
  controls never drawn;
* the Tab. 1-shaped workload (n = 8192, 50 x 50 grid, 5 beta, 10 goals, 96
  controls, T = 2..10) at every horizon;
* the batched plan with a shared control set, per-slot masks changed between
  cycles and a belief reset equals the single-human entry point bit for bit.
"""
import sys

import numpy as np
import pytest
import torch

from paper_2603_01122_amd import scenes

pytestmark = pytest.mark.gpu

SPEEDS6 = np.array([0.25, 0.5, 0.75, 1.0, 1.25, 1.5])


@pytest.fixture(scope="module")
def cap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_01122_amd import capred
    return capred


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def oracle_kw(m, grid, z0, belief, N, H, seed=0, human=0, cycle=0):
    return dict(K=m.K, speed=m.speed, dt=m.dt, beta=m.beta, goals=m.goals, grid=grid, z0=z0,
                belief=belief.reshape(-1), N=N, H=H, seed=seed, human=human, cycle=cycle,
                speeds=m.speeds, speed_mask=m.speed_mask)


def log_close(lb, lb_o):
    """Posterior relative error <= 1e-5: |log b_gpu - log b_oracle| <= 1e-5, every pair."""
    lb, lb_o = np.asarray(lb, np.float64), np.asarray(lb_o, np.float64)
    err = np.max(np.abs(lb - lb_o))
    print(f"max |dlog b| = {err:.3e}")
    return err <= 1e-5


def compare(orc, cap, m, grid, z0, belief, N, H, seed=0, human=0, cycle=0):
    note(f"predict K={m.K} S={m.S} mask={m.speed_mask} N={N} H={H} grid={grid[3]}x{grid[4]}")
    bel = torch.tensor(belief.reshape(m.G, m.B), dtype=torch.float64, device="cuda")
    out = cap.predict_occupancy(m, grid, z0, bel, N, H, seed=seed, human_id=human, cycle=cycle,
                                trace=True)
    torch.cuda.synchronize()
    kw = oracle_kw(m, grid, z0, belief, N, H, seed, human, cycle)
    ref = orc.predict(**kw)
    tk = out["trace_k"].cpu().numpy()
    st, first = orc.tie_check(other_pair=out["trace_pair"].cpu().numpy(), other_k=tk,
                              window=1e-6, **kw)
    assert np.count_nonzero(st == 2) == 0
    allowed = np.repeat([((m.speed_mask or (1 << m.S) - 1) >> s) & 1 == 1 for s in range(m.S)],
                        m.K)
    assert np.all(allowed[tk])
    cg = out["counts"].cpu().numpy().view(np.uint32).astype(np.int64)
    og = out["offgrid"].cpu().numpy().view(np.uint32).astype(np.int64)
    for t in range(H):
        budget = 2 * np.count_nonzero((st == 1) & (first <= t + 1))
        d = np.abs(cg[t] - ref["counts"][t]).sum() + abs(og[t] - int(ref["offgrid"][t]))
        assert d <= budget, (t, d, budget)
        assert 0.5 * d / N <= 1e-3
        assert cg[t].sum() + og[t] == N
    return np.count_nonzero(st == 1)


def test_simulate_tracks_multi_speed(orc, cap):
    K, dt, frame = 16, 0.1, (0.0, 0.0, 0.05)
    r = np.random.default_rng(1)
    n, T = 64, 120
    start = r.uniform(2, 8, (n, 2))
    beta = np.exp(r.uniform(np.log(0.1), np.log(50), n)).astype(np.float32)
    goal = r.uniform(0, 10, (n, 2)).astype(np.float32)
    lat_o, _ = orc.simulate_tracks(K=K, speed=0.0, speeds=SPEEDS6, dt=dt, frame=frame,
                                   start=start, beta=beta, goal=goal, T=T, seed=3, stream=9)
    t = lambda a, dt_: torch.tensor(a, dtype=dt_, device="cuda")
    lat, _ = cap.simulate_tracks(K, 0.0, dt, frame, t(start, torch.float64),
                                 t(beta, torch.float32), t(goal, torch.float32), T, seed=3,
                                 stream_id=9, speeds=SPEEDS6)
    torch.cuda.synchronize()
    assert np.array_equal(lat.cpu().numpy().astype(np.int64), lat_o)


def test_belief_update_multi_speed(orc, cap):
    K, dt = 16, 0.1
    goals = np.array([[8.0, 1.5], [1.0, 8.5], [6.0, 7.0], [9.0, 9.0]], np.float32)
    beta = scenes.BETA_9.copy()
    _, pos = orc.simulate_tracks(K=K, speed=0.0, speeds=SPEEDS6, dt=dt, frame=(0, 0, 0.05),
                                 start=np.array([[3.0, 3.0]]), beta=[3.0], goal=goals[2:3],
                                 T=40, seed=5)
    obs = pos[0]
    m = cap.Model(K, 0.0, dt, beta, goals, speeds=SPEEDS6)
    lb_o, _, _ = orc.belief_update(K=K, speed=0.0, speeds=SPEEDS6, dt=dt, beta=beta,
                                   goals=goals, obs=obs)
    lb = torch.empty((4, beta.size), dtype=torch.float64, device="cuda")
    cap.belief_reset(lb)
    b = torch.empty_like(lb)
    cap.belief_update(m, torch.tensor(obs, device="cuda"), lb, b)
    torch.cuda.synchronize()
    assert log_close(lb.cpu().numpy(), lb_o)


@pytest.mark.parametrize("mask", [0, 0b000011, 0b101000])
def test_predict_96_controls(orc, cap, mask):
    h = scenes.config2().humans[0]
    m = cap.Model(16, 0.0, 0.05, h.beta, h.goals, speeds=SPEEDS6, speed_mask=mask)
    belief = scenes.random_belief(m.G, m.B, seed=3 + mask)
    flagged = compare(orc, cap, m, h.grid, h.start, belief, 40000, 30, seed=mask, human=2,
                      cycle=1)
    print(f"mask {mask}: flagged {flagged}")


def test_predict_multi_speed_shifted_and_k32(orc, cap):
    h = scenes.config2().humans[0]
    beta = np.array([0.05, 3.0, 400.0, 3000.0], np.float32)   # beta * step up to 225
    m = cap.Model(16, 0.0, 0.05, beta, h.goals, speeds=[0.5, 1.5], speed_mask=0)
    compare(orc, cap, m, h.grid, h.start, scenes.random_belief(m.G, m.B, seed=1), 20000, 25,
            seed=7)
    m32 = cap.Model(32, 0.0, 0.05, h.beta, h.goals, speeds=[0.4, 0.8, 1.2, 1.6], speed_mask=0b0110)
    compare(orc, cap, m32, h.grid, h.start, scenes.random_belief(m32.G, m32.B, seed=2), 20000, 25,
            seed=8)


@pytest.mark.parametrize("T", [2, 6, 10])
def test_tab1_shaped_workload(orc, cap, T):
    """n = 8192, 50 x 50 grid, |B| = 5, |G| = 10, |U| = 96 (6 speeds x 16 headings),
    dt = 0.5 s, horizons T = 2..10."""
    r = np.random.default_rng(100 + T)
    cell = 0.1
    goals = r.uniform(0, 5.0, (10, 2)).astype(np.float32)
    beta = np.array([0.1, 0.5, 1.0, 5.0, 10.0], np.float32)
    m = cap.Model(16, 0.0, 0.5, beta, goals, speeds=SPEEDS6)
    belief = scenes.random_belief(10, 5, seed=T)
    compare(orc, cap, m, (0.0, 0.0, cell, 50, 50), (2.5, 2.5), belief, 8192, T, seed=T)


def test_plan_control_set_masks_and_reset(orc, cap):
    from paper_2603_01122_amd.serve import HumanRequest, Server
    sc = scenes.config3()
    hs = sc.humans[:4]
    for h in hs:
        h.N = h.N // 16 + 29
        h.H = 24
    models = {h.hid: cap.Model(16, 0.0, h.dt, h.beta, h.goals, speeds=SPEEDS6,
                               speed_mask=(0b111 if h.hid % 2 else 0)) for h in hs}
    tr = {}
    for h in hs:
        _, pos = orc.simulate_tracks(K=16, speed=0.0, speeds=SPEEDS6, dt=h.dt, frame=h.frame,
                                     start=np.array([h.start]), beta=[h.true_beta],
                                     goal=h.goals[h.true_goal][None], T=6, seed=0, stream=h.hid)
        tr[h.hid] = pos[0]
    srv = Server(16, 0.0, hs[0].dt, len(hs), 24, 256, 256, 6, 9, speeds=SPEEDS6)
    for h in hs:
        srv.submit(HumanRequest(h.hid, models[h.hid], h.grid, h.N, h.H, tr[h.hid][0]))
    note("plan with 96 controls, masks and a belief reset")
    lb = {h.hid: None for h in hs}
    for c in range(5):
        if c == 2:
            srv.plan.set_speed_mask(srv.slot_of[hs[0].hid], 0b000001)
            models[hs[0].hid].speed_mask = 0b000001
        if c == 3:
            srv.plan.reset_belief(srv.slot_of[hs[1].hid])
            lb[hs[1].hid] = None
        srv.step({h.hid: tr[h.hid][c + 1] for h in hs})
        srv.drain()
        torch.cuda.synchronize()
        for h in hs:
            counts, probs, off, post = srv.grids(h.hid, c)
            # posterior: the oracle's update from the last reset
            start = 0 if h.hid != hs[1].hid or c < 3 else 3
            _, b_o, _ = orc.belief_update(K=16, speed=0.0, speeds=SPEEDS6, dt=h.dt, beta=h.beta,
                                          goals=h.goals, obs=tr[h.hid][start:c + 2])
            assert log_close(np.log(post.cpu().numpy()), np.log(b_o)), (c, h.hid)
            single = cap.predict_occupancy(models[h.hid], h.grid, tuple(tr[h.hid][c + 1].astype(float)),
                                           post.contiguous(), h.N, h.H, seed=0, human_id=h.hid,
                                           cycle=c)
            torch.cuda.synchronize()
            assert torch.equal(single["counts"], counts), (c, h.hid)
            assert torch.equal(single["offgrid"], off), (c, h.hid)
    srv.close()


def test_server_stationary_and_goal_departure(orc, cap):
    """The serving loop's detectors: a standing human is predicted with the
    slowest speed only; leaving a goal re-uniformises the belief."""
    from paper_2603_01122_amd.serve import HumanRequest, Server
    h = scenes.config3().humans[0]
    g0 = h.goals[0].astype(np.float64)
    p0 = g0 + [0.1, 0.0]
    obs = [p0, p0 + [0.05, 0.0], p0 + [0.4, 0.0], p0 + [0.4, 0.0], p0 + [0.5, 0.05]]
    obs = [np.asarray(o, np.float32) for o in obs]
    m = cap.Model(16, 0.0, h.dt, h.beta, h.goals, speeds=SPEEDS6)
    srv = Server(16, 0.0, h.dt, 1, 20, 256, 256, 6, 9, speeds=SPEEDS6,
                 stationary=(1e-4, 0b000001), goal_departure=0.3)
    srv.submit(HumanRequest(h.hid, m, h.grid, 5000, 20, obs[0]))
    note("server detectors")
    for c in range(4):
        srv.step({h.hid: obs[c + 1]})
        srv.drain()
        torch.cuda.synchronize()
        counts, _, off, post = srv.grids(h.hid, c)
        start = 1 if c >= 1 else 0          # left the goal at cycle 1 (obs[2])
        _, b_o, _ = orc.belief_update(K=16, speed=0.0, speeds=SPEEDS6, dt=h.dt, beta=h.beta,
                                      goals=h.goals, obs=np.stack(obs[start:c + 2]))
        assert log_close(np.log(post.cpu().numpy()), np.log(b_o)), c
        mask = 0b000001 if c == 2 else 0
        mm = cap.Model(16, 0.0, h.dt, h.beta, h.goals, speeds=SPEEDS6, speed_mask=mask)
        single = cap.predict_occupancy(mm, h.grid, tuple(obs[c + 1].astype(float)),
                                       post.contiguous(), 5000, 20, seed=0, human_id=h.hid,
                                       cycle=c)
        torch.cuda.synchronize()
        assert torch.equal(single["counts"], counts), c
    srv.close()
