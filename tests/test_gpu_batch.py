"""GPU tests of the batched plan and the serving loop.

* batched == per-human reference launches == single-human entry point, bit for
  bit (same kernels' arithmetic, same keys);
* full-size many-human workload (16 humans, 2^14..2^18 particles, H=100) in
  the launch configuration the benchmark times: log posteriors within 1e-5
  of the oracle for every human and pair (posterior relative error 1e-5); histograms within the tie rule for sampled humans;
  counting invariant for every human;
* continuous batching: a human's grids are identical alone and in a changing
  mix; two overlapping streams give the same results as one.
"""
import sys

import numpy as np
import pytest
import torch

from paper_2603_01122_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_01122_amd import capred
    return capred


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def tracks_for(orc, humans, T):
    out = {}
    for h in humans:
        _, pos = orc.simulate_tracks(K=h.K, speed=h.speed, dt=h.dt, frame=h.frame,
                                     start=np.array([h.start]), beta=[h.true_beta],
                                     goal=h.goals[h.true_goal][None], T=T, seed=0, stream=h.hid)
        out[h.hid] = pos[0]
    return out


def small_scene(n=6, N_div=16, H=30):
    sc = scenes.config3()
    hs = sc.humans[:n]
    for h in hs:
        h.N = max(1, h.N // N_div) + 37  # ragged
        h.H = H
    return hs


def make_server(cap, humans, ring=2, n_streams=2, slots=None, max_smooth_radius=0, **tuning):
    from paper_2603_01122_amd.serve import Server
    h0 = humans[0]
    return Server(h0.K, h0.speed, h0.dt, slots or len(humans), max(h.H for h in humans),
                  max(h.grid[3] for h in humans), max(h.grid[4] for h in humans),
                  max(h.G for h in humans), max(h.B for h in humans), ring=ring,
                  n_streams=n_streams, tuning=tuning or None,
                  max_smooth_radius=max_smooth_radius)


def request(cap, h, last, smooth=None):
    from paper_2603_01122_amd.serve import HumanRequest
    return HumanRequest(h.hid, cap.model_of(h), h.grid, h.N, h.H, last, smooth=smooth)


def snapshot(srv, hid, c):
    counts, probs, off, post = srv.grids(hid, c)
    torch.cuda.synchronize()
    return (counts.cpu().numpy().copy(), probs.cpu().numpy().copy(), off.cpu().numpy().copy(),
            post.cpu().numpy().copy())


@pytest.mark.parametrize("shape", [{}, dict(block_threads=256, particles_per_thread=4),
                                   dict(block_threads=512, particles_per_thread=2),
                                   dict(block_threads=256, particles_per_thread=4,
                                        lds_bytes=24576, grid_blocks=768)])
def test_batched_equals_plain_and_single(orc, cap, shape):
    """Batched, per-human and single-human launches give the same bits.  With
    an even number of particles per thread the K = 16 rollout draws two
    particles per pass (their heading chains side by side); the single-human
    entry point draws one particle at a time."""
    humans = small_scene()
    tr = tracks_for(orc, humans, 8)
    note(f"batched vs plain vs single, 6 humans x 4 cycles, shape {shape or 'default'}")
    A = make_server(cap, humans, **shape)
    Bp = make_server(cap, humans, **shape)
    for h in humans:
        A.submit(request(cap, h, tr[h.hid][0]))
        Bp.submit(request(cap, h, tr[h.hid][0]))
    for c in range(4):
        obs = {h.hid: tr[h.hid][c + 1] for h in humans}
        A.step(obs)
        Bp.step(obs, plain=True)
        A.drain()
        Bp.drain()
        for h in humans:
            a = snapshot(A, h.hid, c)
            b = snapshot(Bp, h.hid, c)
            for x, y in zip(a, b):
                assert np.array_equal(x, y), (c, h.hid)
            # the single-human entry point with the plan's posterior and start
            post = torch.tensor(a[3], device="cuda")
            out = cap.predict_occupancy(cap.model_of(h), h.grid, tuple(tr[h.hid][c + 1].astype(float)),
                                        post, h.N, h.H, seed=0, human_id=h.hid, cycle=c)
            torch.cuda.synchronize()
            assert np.array_equal(out["counts"].cpu().numpy(), a[0])
            assert np.array_equal(out["offgrid"].cpu().numpy(), a[2])
            assert np.array_equal(cap.normalize(out["counts"], h.N).cpu().numpy(), a[1])
            assert np.all(a[0].reshape(h.H, -1).sum(1) + a[2] == h.N)
    A.close()
    Bp.close()


@pytest.mark.parametrize("threads,ppt,blocks", [(256, 4, 7), (512, 4, 3), (512, 2, 5),
                                                 (256, 1, 3), (512, 4, 0)])
def test_tile_kinds_cover_every_particle(orc, cap, threads, ppt, blocks):
    """The persistent launch cuts each human into big, half and quarter tiles
    sized from the resident block count; whatever the cut, every particle is
    rolled out once and the grids equal the per-human launches'."""
    humans = small_scene()
    tr = tracks_for(orc, humans, 4)
    note(f"tile kinds: {threads} threads x {ppt}, grid {blocks or 'default'}")
    shape = dict(block_threads=threads, particles_per_thread=ppt, grid_blocks=blocks)
    A = make_server(cap, humans, **shape)
    Bp = make_server(cap, humans, **shape)
    for h in humans:
        A.submit(request(cap, h, tr[h.hid][0]))
        Bp.submit(request(cap, h, tr[h.hid][0]))
    for c in range(2):
        obs = {h.hid: tr[h.hid][c + 1] for h in humans}
        A.step(obs)
        Bp.step(obs, plain=True)
        A.drain()
        Bp.drain()
        for h in humans:
            a = snapshot(A, h.hid, c)
            b = snapshot(Bp, h.hid, c)
            for x, y in zip(a, b):
                assert np.array_equal(x, y), (c, h.hid)
            assert np.all(a[0].reshape(h.H, -1).sum(1) + a[2] == h.N)
    A.close()
    Bp.close()


@pytest.mark.parametrize("lds", [2048, 4096])
def test_window_modes_match_single_human(orc, cap, lds):
    """A small LDS budget drives late steps through the three binning modes
    (two alternating window buffers, both buffers as one, global atomics);
    the counts are exact integers, so they equal the single-human launch's
    (default budget: every step in the first mode)."""
    humans = small_scene(n=3, H=60)
    tr = tracks_for(orc, humans, 3)
    note(f"window modes: lds {lds} B, H=60")
    srv = make_server(cap, humans, block_threads=256, particles_per_thread=2, lds_bytes=lds)
    for h in humans:
        srv.submit(request(cap, h, tr[h.hid][0]))
    for c in range(2):
        srv.step({h.hid: tr[h.hid][c + 1] for h in humans})
        srv.drain()
        for h in humans:
            counts, probs, off, post = snapshot(srv, h.hid, c)
            out = cap.predict_occupancy(cap.model_of(h), h.grid,
                                        tuple(tr[h.hid][c + 1].astype(float)),
                                        torch.tensor(post, device="cuda"), h.N, h.H, seed=0,
                                        human_id=h.hid, cycle=c)
            torch.cuda.synchronize()
            assert np.array_equal(out["counts"].cpu().numpy(), counts), (c, h.hid)
            assert np.array_equal(out["offgrid"].cpu().numpy(), off), (c, h.hid)
    srv.close()


def test_full_size_many_humans_parity(orc, cap):
    sc = scenes.config3()
    humans = sc.humans
    n_pre = 3
    tr = tracks_for(orc, humans, n_pre + 1)
    from paper_2603_01122_amd import tune
    shape = tune.shipped(humans) or {}
    note(f"config3 full size: 16 humans, 3 cycles, launch shape {shape}")
    srv = make_server(cap, humans, **shape)
    for h in humans:
        srv.submit(request(cap, h, tr[h.hid][0]))
    for c in range(n_pre):
        srv.step({h.hid: tr[h.hid][c + 1] for h in humans})
    srv.drain()
    c = n_pre - 1
    snaps = {h.hid: snapshot(srv, h.hid, c) for h in humans}
    for h in humans:
        counts, probs, off, post = snaps[h.hid]
        assert np.all(counts.reshape(h.H, -1).sum(1) + off == h.N)
        lb_o, b_o, _ = orc.belief_update(K=h.K, speed=h.speed, dt=h.dt, beta=h.beta,
                                         goals=h.goals, obs=tr[h.hid][:n_pre + 1])
        assert np.max(np.abs(np.log(post) - lb_o)) <= 1e-5, h.hid
    # histogram parity under the tie rule for the smallest and a mid-size human.
    # The oracle predicts from its own posterior; the GPU's posterior agrees to
    # 1e-5 in log, so its pair-CDF boundaries agree to 1e-5 (pair window).
    order = sorted(humans, key=lambda h: h.N)
    for h in (order[0], order[len(order) // 2]):
        counts, probs, off, post = snaps[h.hid]
        z0 = tuple(tr[h.hid][n_pre].astype(float))
        note(f"oracle human {h.hid} N={h.N}")
        single = cap.predict_occupancy(cap.model_of(h), h.grid, z0,
                                       torch.tensor(post, device="cuda"), h.N, h.H, seed=0,
                                       human_id=h.hid, cycle=c, trace=True)
        torch.cuda.synchronize()
        assert np.array_equal(single["counts"].cpu().numpy(), counts)
        _, b_o, _ = orc.belief_update(K=h.K, speed=h.speed, dt=h.dt, beta=h.beta, goals=h.goals,
                                      obs=tr[h.hid][:n_pre + 1])
        kw = dict(K=h.K, speed=h.speed, dt=h.dt, beta=h.beta, goals=h.goals, grid=h.grid,
                  z0=z0, belief=b_o.reshape(-1), N=h.N, H=h.H, seed=0, human=h.hid, cycle=c)
        ref = orc.predict(**kw)
        st, first = orc.tie_check(other_pair=single["trace_pair"].cpu().numpy(),
                                  other_k=single["trace_k"].cpu().numpy(), window=1e-6,
                                  pair_window=1e-5, **kw)
        assert np.count_nonzero(st == 2) == 0
        for t in range(h.H):
            budget = 2 * np.count_nonzero((st == 1) & (first <= t + 1))
            d = np.abs(counts[t].astype(np.int64) - ref["counts"][t]).sum() + \
                abs(int(off[t]) - int(ref["offgrid"][t]))
            assert d <= budget
            assert 0.5 * d / h.N <= 1e-3
        print(f"human {h.hid}: flagged {np.count_nonzero(st == 1)} of {h.N}")
    srv.close()


def _trace_histogram(orc, h, z0, trace_k):
    """Per-step histogram of the lattice paths of the given headings [N, H]."""
    x0, y0, cell, nx, ny = h.grid
    Sx, Sy = orc.lattice_steps(h.K, h.speed, h.dt, cell)
    q = cell / 65536.0
    X = np.full(trace_k.shape[0], np.rint((z0[0] - x0) / q), np.int64)
    Y = np.full(trace_k.shape[0], np.rint((z0[1] - y0) / q), np.int64)
    Sx, Sy = Sx.astype(np.int64), Sy.astype(np.int64)
    counts = np.zeros((h.H, ny * nx), np.int64)
    off = np.zeros(h.H, np.int64)
    for t in range(h.H):
        k = trace_k[:, t]
        X += Sx[k]
        Y += Sy[k]
        cx, cy = X >> 16, Y >> 16
        inside = (cx >= 0) & (cx < nx) & (cy >= 0) & (cy < ny)
        counts[t] = np.bincount((cy[inside] * nx + cx[inside]), minlength=ny * nx)
        off[t] = np.count_nonzero(~inside)
    return counts.reshape(h.H, ny, nx), off


def test_long_run_all_humans_parity(orc, cap):
    """The 16-human serving workload at full size in the benchmark's launch
    shape, served for 300 cycles (one new observed step per human per cycle):
    * every human's log posterior equals the oracle's update over its whole
      observed history within 1e-5 for every pair, at cycles 1, 100, 200, 300;
    * at the last cycle, for all 16 humans: the batched grids equal the
      single-human entry point's, equal the histogram rebuilt on the host from
      its per-particle trace, and 4096 sampled particles per human agree with
      the oracle (fed the oracle's own posterior) under the tie rule."""
    from paper_2603_01122_amd import tune
    sc = scenes.config3()
    humans = sc.humans
    n_cycles, sample = 300, 4096
    tr = tracks_for(orc, humans, n_cycles)
    shape = tune.shipped(humans) or {}
    note(f"config3 long run: 16 humans, {n_cycles} cycles, launch shape {shape}")
    srv = make_server(cap, humans, **shape)
    for h in humans:
        srv.submit(request(cap, h, tr[h.hid][0]))
    worst = 0.0
    for c in range(n_cycles):
        srv.step({h.hid: tr[h.hid][c + 1] for h in humans})
        if c + 1 in (1, 100, 200, n_cycles):
            srv.drain()
            torch.cuda.synchronize()
            note(f"posteriors after {c + 1} cycles")
            for h in humans:
                lb_o, _, _ = orc.belief_update(K=h.K, speed=h.speed, dt=h.dt, beta=h.beta,
                                               goals=h.goals, obs=tr[h.hid][:c + 2])
                err = np.max(np.abs(srv.log_belief(h.hid).cpu().numpy() - lb_o))
                worst = max(worst, err)
                assert err <= 1e-5, (c, h.hid, err)
    print(f"max |dlog b| over 300 cycles: {worst:.3e}")
    c = n_cycles - 1
    r = np.random.default_rng(17)
    flagged = 0
    for h in humans:
        counts, probs, off, post = srv.grids(h.hid, c)
        z0 = tuple(tr[h.hid][c + 1].astype(float))
        note(f"human {h.hid} N={h.N}: single-human trace, host histogram, oracle sample")
        single = cap.predict_occupancy(cap.model_of(h), h.grid, z0, post.contiguous(), h.N, h.H,
                                       seed=0, human_id=h.hid, cycle=c, trace=True)
        torch.cuda.synchronize()
        assert torch.equal(single["counts"], counts), h.hid
        assert torch.equal(single["offgrid"], off), h.hid
        tk = single["trace_k"].cpu().numpy()
        tp = single["trace_pair"].cpu().numpy()
        del single
        hc, ho = _trace_histogram(orc, h, z0, tk)
        assert np.array_equal(counts.cpu().numpy().view(np.uint32).astype(np.int64), hc), h.hid
        assert np.array_equal(off.cpu().numpy().astype(np.int64), ho), h.hid
        _, b_o, _ = orc.belief_update(K=h.K, speed=h.speed, dt=h.dt, beta=h.beta,
                                      goals=h.goals, obs=tr[h.hid][:c + 2])
        idx = np.sort(r.choice(h.N, sample, replace=False))
        kw = dict(K=h.K, speed=h.speed, dt=h.dt, beta=h.beta, goals=h.goals, grid=h.grid,
                  z0=z0, belief=b_o.reshape(-1), N=h.N, H=h.H, seed=0, human=h.hid, cycle=c,
                  idx=idx)
        st, _ = orc.tie_check(other_pair=tp[idx], other_k=tk[idx], window=1e-6,
                              pair_window=1e-9, **kw)
        assert np.count_nonzero(st == 2) == 0, h.hid
        assert np.count_nonzero(st == 1) <= 1e-3 * sample, h.hid
        flagged += np.count_nonzero(st == 1)
    print(f"sampled particles at CDF ties: {flagged} of {16 * sample}")
    srv.close()


def test_union_in_cycle(orc, cap):
    """The union stage inside the cycle (Sec. IV-B point-wise maximum): every
    cycle's union grid equals the oracle's maximum over the probability grids of
    the humans that share the union's frame (steps beyond a human's horizon
    count as 0), excluding a human on another grid; one member has smoothed
    probabilities; batched and per-human launches give the same bits, and a
    replay of the rollout leaves the union alone."""
    humans = small_scene(n=5, N_div=8, H=20)
    humans[1].H = 14
    humans[3].grid = (humans[3].grid[0], humans[3].grid[1], humans[3].grid[2],
                      humans[3].grid[3], 200)          # another frame: not in the union
    frame, uH = humans[0].grid, 20
    tr = tracks_for(orc, humans, 5)
    sm = {humans[2].hid: (1.0, 2)}
    note("union of 4 of 5 humans inside the cycle, batched and plain, 3 cycles")
    from paper_2603_01122_amd.serve import Server
    h0 = humans[0]
    mk = lambda: Server(h0.K, h0.speed, h0.dt, len(humans), 20, 256, 256, max(h.G for h in humans),
                        9, max_smooth_radius=2, union=(frame, uH))
    A, Bp = mk(), mk()
    for h in humans:
        A.submit(request(cap, h, tr[h.hid][0], smooth=sm.get(h.hid)))
        Bp.submit(request(cap, h, tr[h.hid][0], smooth=sm.get(h.hid)))
    for c in range(3):
        obs = {h.hid: tr[h.hid][c + 1] for h in humans}
        A.step(obs)
        Bp.step(obs, plain=True)
        A.drain()
        Bp.drain()
        torch.cuda.synchronize()
        members = []
        for h in humans:
            if h.hid == humans[3].hid:
                continue
            probs = snapshot(A, h.hid, c)[1]
            padded = np.zeros((uH,) + probs.shape[1:], np.float32)
            padded[:h.H] = probs
            members.append(padded)
        ref = orc.union_max(members)
        got = A.union_grid(c).cpu().numpy()
        assert np.array_equal(got, ref), c
        assert np.array_equal(Bp.union_grid(c).cpu().numpy(), ref), c
        assert np.count_nonzero(ref[humans[1].H:]) > 0
    A.plan.replay_rollout()
    torch.cuda.synchronize()
    assert np.array_equal(A.union_grid(2).cpu().numpy(), ref)
    A.close()
    Bp.close()


def test_continuous_batching_invariance(orc, cap):
    humans = small_scene(n=5, N_div=8, H=25)
    tr = tracks_for(orc, humans, 12)
    x = humans[2]
    note("alone vs churning mix")
    alone = make_server(cap, [x], slots=1)
    alone.submit(request(cap, x, tr[x.hid][0]))
    mix = make_server(cap, humans, slots=3)  # fewer slots than humans: some wait
    mix.submit(request(cap, humans[0], tr[humans[0].hid][0]))
    mix.submit(request(cap, x, tr[x.hid][0]))
    got_alone, got_mix = [], []
    for c in range(8):
        if c == 2:
            mix.submit(request(cap, humans[1], tr[humans[1].hid][c]))
            mix.submit(request(cap, humans[3], tr[humans[3].hid][c]))  # waits for a slot
        if c == 4:
            mix.depart(humans[0].hid)                                  # frees a slot
        if c == 6:
            mix.depart(humans[1].hid)
            mix.submit(request(cap, humans[4], tr[humans[4].hid][c]))
        alone.step({x.hid: tr[x.hid][c + 1]})
        mix.step({h.hid: tr[h.hid][c + 1] for h in humans})
        alone.drain()
        mix.drain()
        got_alone.append(snapshot(alone, x.hid, c))
        got_mix.append(snapshot(mix, x.hid, c))
    assert humans[3].hid in mix.slot_of and humans[4].hid in mix.slot_of
    for a, b in zip(got_alone, got_mix):
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
    alone.close()
    mix.close()


def test_churn_with_cycles_in_flight_matches_alone(orc, cap):
    """Humans with different goal counts, horizons and grids leave and arrive
    while the previous cycle is still on the device (two cycles in flight, no
    drain in between); a departed human's slot is reused only after its cycles
    complete.  Every human's counts, probabilities, off-grid counts and
    posterior at every cycle it was served equal those of the same human served
    alone with the same observations and cycle numbers."""
    humans = scenes.config3().humans[:5]
    for h, H, ny in zip(humans, (30, 12, 26, 10, 22), (256, 200, 256, 180, 224)):
        h.N = h.N // 16 + 41
        h.H = H
        h.grid = (h.grid[0], h.grid[1], h.grid[2], h.grid[3], ny)
    tr = tracks_for(orc, humans, 12)
    n_cycles = 10
    note("churn with two cycles in flight: 3 slots, 5 humans of different G, H, grids")
    mix = make_server(cap, humans, slots=3)
    submitted = {}

    def submit(h, c):
        mix.submit(request(cap, h, tr[h.hid][c]))
        submitted[h.hid] = c

    for h in humans[:3]:
        submit(h, 0)
    got = {h.hid: {} for h in humans}
    for c in range(n_cycles):
        if c == 3:                      # cycle 2 still in flight
            mix.depart(humans[0].hid)
            submit(humans[3], c)
        if c == 5:                      # cycle 4 still in flight
            mix.depart(humans[2].hid)
            submit(humans[4], c)
        mix.step({h.hid: tr[h.hid][c + 1] for h in humans})
        if c % 2 == 1:
            mix.drain()
            for cc in (c - 1, c):
                for hid in mix.records[cc].humans:
                    if hid in mix.slot_of:
                        got[hid][cc] = snapshot(mix, hid, cc)
    mix.close()
    served = {h.hid: [r.cycle for r in mix.records if h.hid in r.humans] for h in humans}
    assert all(served[h.hid] for h in humans)
    for h in humans:
        c0, c1 = served[h.hid][0], served[h.hid][-1]
        assert served[h.hid] == list(range(c0, c1 + 1))
        assert got[h.hid], h.hid
        note(f"human {h.hid} alone, cycles {c0}..{c1}")
        alone = make_server(cap, [h], slots=1)
        for c in range(c0):
            alone.step({})
        alone.submit(request(cap, h, tr[h.hid][submitted[h.hid]]))
        for c in range(c0, c1 + 1):
            alone.step({h.hid: tr[h.hid][c + 1]})
            alone.drain()
            if c in got[h.hid]:
                ref = snapshot(alone, h.hid, c)
                for u, v in zip(ref, got[h.hid][c]):
                    assert np.array_equal(u, v), (h.hid, c)
        alone.close()


def test_shifted_human_in_a_mix_matches_alone(orc, cap):
    """One human's beta grid reaches beta v dt = 96 > 80, so its draws need the
    max-shifted exponent (a separately compiled rollout variant).  The mixed
    launch then runs that variant; the other humans' tiles take the unshifted
    body inside it, so every human's grids and posterior equal those of the
    same human served alone, bit for bit."""
    humans = small_scene(n=4, N_div=16, H=20)
    humans[1].beta = np.array([0.5, 50.0, 4000.0], np.float32)
    tr = tracks_for(orc, humans, 5)
    note("shifted-exponent human in a mix of 4 vs each alone, 3 cycles")
    mix = make_server(cap, humans)
    for h in humans:
        mix.submit(request(cap, h, tr[h.hid][0]))
    got = {h.hid: [] for h in humans}
    for c in range(3):
        mix.step({h.hid: tr[h.hid][c + 1] for h in humans})
        mix.drain()
        for h in humans:
            got[h.hid].append(snapshot(mix, h.hid, c))
    mix.close()
    for h in humans:
        alone = make_server(cap, [h], slots=1)
        alone.submit(request(cap, h, tr[h.hid][0]))
        for c in range(3):
            alone.step({h.hid: tr[h.hid][c + 1]})
            alone.drain()
            for u, v in zip(snapshot(alone, h.hid, c), got[h.hid][c]):
                assert np.array_equal(u, v), (h.hid, c)
        alone.close()


def test_resume_from_carried_state(orc, cap):
    """Checkpoint / resume of a served human: its carried state is the log
    posterior, the last observed position and the cycle number (the random
    streams are keyed by human id, cycle and seed).  A new server that starts
    at that cycle with that state reproduces the uninterrupted run bit for
    bit, in a different slot and mix."""
    humans = small_scene(n=3, N_div=16, H=20)
    x = humans[1]
    tr = tracks_for(orc, humans, 12)
    note("resume a human from its log posterior, last position and cycle")
    A = make_server(cap, humans)
    for h in humans:
        A.submit(request(cap, h, tr[h.hid][0]))
    ref, lb6 = {}, None
    for c in range(10):
        A.step({h.hid: tr[h.hid][c + 1] for h in humans})
        A.drain()
        if c == 5:
            lb6 = A.log_belief(x.hid).cpu().numpy().copy()
        if c >= 6:
            ref[c] = snapshot(A, x.hid, c)
    A.close()
    from paper_2603_01122_amd.serve import HumanRequest, Server
    B = Server(x.K, x.speed, x.dt, 2, x.H, 256, 256, 6, 9, first_cycle=6)
    other = humans[2]
    B.submit(request(cap, other, tr[other.hid][5]))     # takes slot 0: x lands in slot 1
    B.submit(HumanRequest(x.hid, cap.model_of(x), x.grid, x.N, x.H, tr[x.hid][6],
                          log_belief=lb6))
    for c in range(6, 10):
        B.step({x.hid: tr[x.hid][c + 1], other.hid: tr[other.hid][c]})
        B.drain()
        assert B.slot_of[x.hid] == 1
        for u, v in zip(snapshot(B, x.hid, c), ref[c]):
            assert np.array_equal(u, v), c
    B.close()


def test_two_streams_overlap_equals_one(orc, cap):
    humans = small_scene(n=4, N_div=4, H=40)
    tr = tracks_for(orc, humans, 10)
    note("ring 2 / two streams vs ring 1 / one stream")
    one = make_server(cap, humans, ring=1, n_streams=1)
    two = make_server(cap, humans, ring=2, n_streams=2)
    for s in (one, two):
        for h in humans:
            s.submit(request(cap, h, tr[h.hid][0]))
    res1, res2 = [], []
    for c in range(6):
        obs = {h.hid: tr[h.hid][c + 1] for h in humans}
        one.step(obs)
        one.drain()
        res1.append([snapshot(one, h.hid, c) for h in humans])
        two.step(obs)
        if c % 2 == 1:  # two cycles in flight before reading
            two.drain()
            res2.append([snapshot(two, h.hid, c - 1) for h in humans])
            res2.append([snapshot(two, h.hid, c) for h in humans])
    for a, b in zip(res1, res2):
        for x, y in zip(a, b):
            for u, v in zip(x, y):
                assert np.array_equal(u, v)
    one.close()
    two.close()


def test_batched_smoothing(orc, cap):
    """Slots asking for Gaussian-smoothed probabilities (the smoothing stage in
    the cycle's graph) get exactly cap_smooth_occupancy of their counts, in the
    batched and in the per-human launch; the others keep count / N; the
    smoothed grids agree with the oracle's direct sum within (4r + 6) 2^-24."""
    humans = small_scene(n=5, N_div=8, H=20)
    tr = tracks_for(orc, humans, 4)
    sm = {humans[0].hid: (1.0, 3), humans[2].hid: (2.0, 6), humans[3].hid: (0.8, 1)}
    note("batched smoothing, 5 humans (3 smoothed), 3 cycles")
    A = make_server(cap, humans, max_smooth_radius=6)
    Bp = make_server(cap, humans, max_smooth_radius=6)
    for h in humans:
        A.submit(request(cap, h, tr[h.hid][0], smooth=sm.get(h.hid)))
        Bp.submit(request(cap, h, tr[h.hid][0], smooth=sm.get(h.hid)))
    for c in range(3):
        obs = {h.hid: tr[h.hid][c + 1] for h in humans}
        A.step(obs)
        Bp.step(obs, plain=True)
        A.drain()
        Bp.drain()
        for h in humans:
            a = snapshot(A, h.hid, c)
            b = snapshot(Bp, h.hid, c)
            for x, y in zip(a, b):
                assert np.array_equal(x, y), (c, h.hid)
            counts = torch.tensor(a[0], device="cuda")
            if h.hid in sm:
                sigma, r = sm[h.hid]
                ref = cap.smooth_occupancy(counts, h.N, sigma, r)
                torch.cuda.synchronize()
                assert np.array_equal(ref.cpu().numpy(), a[1])
                if c == 2:
                    o = orc.smooth(a[0].view(np.uint32), h.N, sigma, r)
                    assert np.all(np.abs(a[1] - o) <= (4 * r + 6) * 2.0 ** -24 * o)
            else:
                assert np.array_equal(cap.normalize(counts, h.N).cpu().numpy(), a[1])
    A.close()
    Bp.close()
    p = cap.Plan(16, 1.2, 0.02, 1, max_obs=1, max_smooth_radius=2)
    h = humans[0]
    buf = cap.SlotBuffers.allocate(cap.model_of(h), h.grid, 5, 2)
    with pytest.raises(cap.CapError):
        p.admit(0, 1, cap.model_of(h), h.grid, 100, 5, h.start, buf, smooth=(1.0, 3))
    with pytest.raises(cap.CapError):
        p.admit(0, 1, cap.model_of(h), h.grid, 100, 5, h.start, buf, smooth=(0.0, 2))
    p.close()
    with pytest.raises(cap.CapError):
        cap.Plan(16, 1.2, 0.02, 1, max_smooth_radius=17)


def test_plan_errors(cap):
    p = cap.Plan(16, 1.2, 0.02, 2, max_obs=1)
    h = scenes.config3().humans[0]
    buf = cap.SlotBuffers.allocate(cap.model_of(h), h.grid, 5, 2)
    p.admit(0, 1, cap.model_of(h), h.grid, 100, 5, h.start, buf)
    with pytest.raises(cap.CapError):
        p.admit(0, 2, cap.model_of(h), h.grid, 100, 5, h.start, buf)   # occupied
    p.stage(0, [h.start])
    with pytest.raises(cap.CapError):
        p.stage(0, [h.start])                                          # > max_obs
    with pytest.raises(cap.CapError):
        p.stage(1, [h.start])                                          # empty slot
    with pytest.raises(cap.CapError):
        p.run(0, 0x7FFFFFFF)
    p.run(0, 0)
    p.sync()
    p.close()


def test_stage_many_is_all_or_nothing(cap):
    """Batched staging validates every entry before staging any: a call with
    one bad entry leaves the good slots unstaged, so that the same positions
    can be staged again."""
    p = cap.Plan(16, 1.2, 0.02, 3, max_obs=1)
    h = scenes.config3().humans[0]
    bufs = [cap.SlotBuffers.allocate(cap.model_of(h), h.grid, 5, 2) for _ in range(2)]
    p.admit(0, 1, cap.model_of(h), h.grid, 100, 5, h.start, bufs[0])
    p.admit(1, 2, cap.model_of(h), h.grid, 100, 5, h.start, bufs[1])
    with pytest.raises(cap.CapError):
        p.stage_many([0, 2], [h.start, h.start])                       # slot 2 is empty
    with pytest.raises(cap.CapError):
        p.stage_many([0, 0], [h.start, h.start])                       # > max_obs for slot 0
    with pytest.raises(cap.CapError):
        p.stage_many([1, 0], [h.start, (float("nan"), 0.0)])           # bad position
    p.stage_many([0, 1], [h.start, h.start])                           # nothing was staged before
    with pytest.raises(cap.CapError):
        p.stage(0, [h.start])                                          # now full
    p.run(0, 0)
    p.sync()
    p.close()


def test_replay_reproduces_the_cycle(orc, cap):
    """Re-running the latest rollout alone (the benchmark's kernel timing)
    recomputes the same grids: the clear covers both the previous and the new
    reach windows."""
    humans = small_scene(n=4, N_div=8, H=30)
    tr = tracks_for(orc, humans, 6)
    srv = make_server(cap, humans)
    for h in humans:
        srv.submit(request(cap, h, tr[h.hid][0]))
    note("replay of the latest rollout")
    for c in range(4):
        srv.step({h.hid: tr[h.hid][c + 1] for h in humans})
    srv.drain()
    torch.cuda.synchronize()
    before = {h.hid: snapshot(srv, h.hid, 3) for h in humans}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    e1.record()
    for _ in range(3):
        srv.plan.replay_rollout(torch.cuda.current_stream(), e0, e1)
    torch.cuda.synchronize()
    for h in humans:
        after = snapshot(srv, h.hid, 3)
        assert np.array_equal(after[0], before[h.hid][0])
        assert np.array_equal(after[2], before[h.hid][2])
    srv.close()
