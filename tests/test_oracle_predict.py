"""Pins for the oracle's Alg. 1 (particle prediction), none of which reuses the
oracle's own code path:

* K=4 closed form: from x=0 toward g=(D,0) the four next-state distances are
  D-s, sqrt(D^2+s^2), D+s, sqrt(D^2+s^2); every particle's first heading must be
  the inverse-CDF choice of those hand-derived weights with the u that
  PyTorch's Philox engine gives for the documented counter.
* beta -> 0: headings are uniform (Eq. human_softmax_policy as beta -> 0), so
  the choice is exactly floor(u K).
* beta -> inf: the policy is the argmax; every particle follows the greedy
  path toward its goal, computed here by brute force.
* exact enumeration of Eq. (human_prediction)/(human_prediction_multi_step)
  over all K^H heading paths and all pairs, against the oracle's Monte Carlo
  (chi-square), and the H=1 multinomial z-scores.
* pair draws: the pair index is the inverse CDF of the belief at u from the
  documented pair counter, and pair frequencies follow the belief.
* counting invariant: counts + off-grid = N at every step.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.stats

from paper_2603_01122_amd import scenes


def u_of(torch_philox, seed, c0, c1, c2, c3, word):
    w = torch_philox(seed, c0, c1, c2, c3)[word]
    return ((int(w) >> 9) * 2 + 1) * 2.0 ** -24


def test_lattice_steps_closed_form(orc):
    # K=4, v*dt = 0.1 m, cell 0.1 m -> q = 0.1/65536, step = 65536 lattice units
    Sx, Sy = orc.lattice_steps(4, 1.0, 0.1, 0.1)
    assert list(Sx) == [65536, 0, -65536, 0] and list(Sy) == [0, 65536, 0, -65536]
    Sx, Sy = orc.lattice_steps(8, 1.2, 0.05, 0.05)   # step 0.06 m = 1.2 cells
    r = round(0.06 / (0.05 / 65536))
    d = round(0.06 / math.sqrt(2) / (0.05 / 65536))
    assert list(Sx) == [r, d, 0, -d, -r, -d, 0, d]
    assert list(Sy) == [0, d, r, d, 0, -d, -r, -d]


@pytest.mark.parametrize("axis", [0, 1])
def test_k4_closed_form_first_step(orc, torch_philox, axis):
    K, v, dt, cell = 4, 1.0, 0.1, 0.1
    s = v * dt
    D = 1.7
    beta = np.array([2.5], np.float32)
    goal = np.zeros((1, 2), np.float32)
    goal[0, axis] = D
    grid = (-3.2, -3.2, cell, 64, 64)
    # z0 = (0,0) sits on the lattice; goal D=1.7 is a multiple of q? use exact lattice
    N, H, seed, hid, cyc = 3000, 1, 11, 3, 5
    out = orc.predict(K=K, speed=v, dt=dt, beta=beta, goals=goal, grid=grid, z0=(0.0, 0.0),
                      belief=np.ones(1), N=N, H=H, seed=seed, human=hid, cycle=cyc, trace=True)
    q = cell / 65536
    Dq = round((float(np.float32(D)) + 3.2) / q) * q - round(3.2 / q) * q  # lattice goal distance
    d_par = [Dq - s, math.hypot(Dq, s), Dq + s, math.hypot(Dq, s)]
    if axis == 1:
        d_par = [math.hypot(Dq, s), Dq - s, math.hypot(Dq, s), Dq + s]
    w = np.exp(-float(beta[0]) * (np.array(d_par) - min(d_par)))
    cdf = np.cumsum(w)
    ks = []
    for i in range(N):
        u = u_of(torch_philox, seed, i, 0, hid, 2 * cyc + 1, 0)
        ks.append(int(np.argmax(u * cdf[-1] < cdf)))
    assert np.array_equal(out["trace_k"][:, 0], np.array(ks, np.uint8))
    # heading toward the goal is the most likely one
    freq = np.bincount(out["trace_k"][:, 0], minlength=4) / N
    assert np.argmax(freq) == (0 if axis == 0 else 1)


def test_beta_to_zero_uniform_headings(orc, torch_philox):
    sc = scenes.config1()
    h = sc.humans[0]
    beta = np.full(3, 1e-12, np.float32)
    N, H = 500, 9
    out = orc.predict(K=h.K, speed=h.speed, dt=h.dt, beta=beta, goals=h.goals, grid=h.grid,
                      z0=h.start, belief=np.full(h.G * 3, 1.0 / (h.G * 3)), N=N, H=H, seed=0,
                      human=7, cycle=2, trace=True)
    for i in range(0, N, 7):
        for t in range(1, H + 1):
            u = u_of(torch_philox, 0, i, (t - 1) // 4, 7, 5, (t - 1) % 4)
            assert out["trace_k"][i, t - 1] == math.floor(u * h.K), (i, t)


def test_beta_to_inf_greedy_paths(orc):
    K, v, dt, cell = 8, 1.0, 0.1, 0.1
    goals = np.array([[5.13, 1.37], [0.71, 4.46]], np.float32)
    grid = (0.0, 0.0, cell, 64, 64)
    z0 = (3.03, 2.91)
    beta = np.array([1e6], np.float32)
    belief = np.array([0.3, 0.7])
    N, H = 2000, 25
    out = orc.predict(K=K, speed=v, dt=dt, beta=beta, goals=goals, grid=grid, z0=z0,
                      belief=belief, N=N, H=H, seed=4, trace=True)
    q = cell / 65536
    th = 2 * np.pi * np.arange(K) / K
    S = np.stack([np.rint(v * dt * np.cos(th) / q), np.rint(v * dt * np.sin(th) / q)], 1)
    P0 = np.rint((np.array(z0) - 0.0) / q)
    expect = {}
    for g in range(2):
        Gl = np.rint((goals[g].astype(np.float64) - 0.0) / q)
        p = P0.copy()
        ks, cells = [], []
        for t in range(H):
            dist = np.hypot(*((p + S - Gl) * q).T)
            k = int(np.argmin(dist))
            assert np.sort(dist)[1] - dist[k] > 1e-9  # no exact tie in this scene
            p = p + S[k]
            ks.append(k)
            cx, cy = int(np.floor(p[0] / 65536)), int(np.floor(p[1] / 65536))
            cells.append(cy * 64 + cx)
        expect[g] = (np.array(ks, np.uint8), np.array(cells))
    ng = np.zeros(2, int)
    for i in range(N):
        g = out["trace_pair"][i]
        ng[g] += 1
        assert np.array_equal(out["trace_k"][i], expect[g][0])
        assert np.array_equal(out["trace_cell"][i], expect[g][1])
    # grid = sum_g N_g * delta(greedy path)
    for t in range(H):
        ref = np.zeros(64 * 64, np.int64)
        for g in range(2):
            ref[expect[g][1][t]] += ng[g]
        assert np.array_equal(out["counts"][t].reshape(-1).astype(np.int64), ref)


def test_pair_draws_follow_belief(orc, torch_philox):
    G, B = 3, 4
    belief = scenes.random_belief(G, B, seed=3, sparsity=0.3)
    beta = np.array([0.1, 1, 10, 100], np.float32)
    goals = np.array([[1, 1], [2, 5], [5, 2]], np.float32)
    N = 20000
    out = orc.predict(K=8, speed=1.0, dt=0.1, beta=beta, goals=goals,
                      grid=(0, 0, 0.1, 64, 64), z0=(3.2, 3.2), belief=belief, N=N, H=1, seed=9,
                      human=2, cycle=1, trace=True)
    P = np.cumsum(belief.reshape(-1))
    for i in range(0, N, 97):
        u = u_of(torch_philox, 9, i, 0, 2, 2, 0)
        j = int(np.searchsorted(P, u, side="right"))
        if j >= P.size:
            j = int(np.nonzero(belief.reshape(-1) > 0)[0][-1])
        assert out["trace_pair"][i] == j
    cnt = np.bincount(out["trace_pair"], minlength=G * B)
    nz = belief.reshape(-1) > 0
    assert np.all(cnt[~nz] == 0)
    chi = scipy.stats.chisquare(cnt[nz], N * belief.reshape(-1)[nz] / belief.sum())
    assert chi.pvalue > 1e-4


def _exact_distribution(K, v, dt, cell, beta, goals, belief, z0, H, nx, ny):
    """Exact per-step cell distribution: enumerate every heading path for every
    (beta, g) pair and multiply the Boltzmann probabilities along it."""
    q = cell / 65536
    th = 2 * np.pi * np.arange(K) / K
    S = np.stack([np.rint(v * dt * np.cos(th) / q), np.rint(v * dt * np.sin(th) / q)], 1)
    P0 = np.rint(np.asarray(z0, np.float64) / q)
    dist = np.zeros((H, ny * nx + 1))       # last bin: off grid
    G, B = goals.shape[0], beta.size
    for g in range(G):
        Gl = np.rint(goals[g].astype(np.float64) / q)
        for b in range(B):
            pb = belief[g * B + b]
            if pb == 0:
                continue
            for path in itertools.product(range(K), repeat=H):
                p = P0.copy()
                prob = pb
                cells = []
                for t, k in enumerate(path):
                    Qk = -np.hypot(*((p + S - Gl) * q).T)
                    pi = np.exp(float(beta[b]) * (Qk - Qk.max()))
                    prob *= pi[k] / pi.sum()
                    p = p + S[k]
                    cx, cy = int(np.floor(p[0] / 65536)), int(np.floor(p[1] / 65536))
                    cells.append(cy * nx + cx if (0 <= cx < nx and 0 <= cy < ny) else ny * nx)
                # the marginal at step t sums whole-path probabilities (Chapman-Kolmogorov)
                for t, c in enumerate(cells):
                    dist[t, c] += prob
    return dist


@pytest.mark.parametrize("K,H", [(4, 4), (8, 3)])
def test_enumeration_matches_monte_carlo(orc, K, H):
    v, dt, cell, nx, ny = 1.0, 0.1, 0.05, 16, 16
    beta = np.array([0.5, 3.0, 20.0], np.float32)
    goals = np.array([[0.61, 0.13], [0.09, 0.47]], np.float32)
    belief = np.array([0.1, 0.2, 0.15, 0.25, 0.2, 0.1])
    z0 = (0.4137, 0.3862)
    exact = _exact_distribution(K, v, dt, cell, beta, goals, belief, z0, H, nx, ny)
    assert np.allclose(exact.sum(1), 1.0)
    N = 400000
    out = orc.predict(K=K, speed=v, dt=dt, beta=beta, goals=goals, grid=(0, 0, cell, nx, ny),
                      z0=z0, belief=belief, N=N, H=H, seed=21)
    for t in range(H):
        mc = np.concatenate([out["counts"][t].reshape(-1), [out["offgrid"][t]]]).astype(float)
        e = exact[t] * N
        keep = e >= 5
        obs = np.append(mc[keep], mc[~keep].sum())
        exp_ = np.append(e[keep], e[~keep].sum())
        if exp_[-1] < 5:
            obs[-2] += obs[-1]
            exp_[-2] += exp_[-1]
            obs, exp_ = obs[:-1], exp_[:-1]
        assert abs(mc[~keep].sum() - e[~keep].sum()) < 6 * math.sqrt(max(e[~keep].sum(), 1))
        p = scipy.stats.chisquare(obs, exp_ * obs.sum() / exp_.sum()).pvalue
        assert p > 1e-4, (t, p)
        tv = 0.5 * np.abs(mc / N - exact[t]).sum()
        assert tv < 3 * math.sqrt(np.count_nonzero(exact[t]) / N)


def test_one_step_multinomial(orc):
    K, v, dt, cell = 16, 1.2, 0.05, 0.05
    beta = scenes.BETA_9
    goals = np.array([[1.0, 9.0], [11.0, 4.0], [6.3, 6.8]], np.float32)
    belief = scenes.random_belief(3, 9, seed=5)
    z0 = (6.4012, 6.3991)
    N = 200000
    out = orc.predict(K=K, speed=v, dt=dt, beta=beta, goals=goals, grid=(0, 0, cell, 256, 256),
                      z0=z0, belief=belief.reshape(-1), N=N, H=1, seed=1)
    q = cell / 65536
    th = 2 * np.pi * np.arange(K) / K
    S = np.stack([np.rint(v * dt * np.cos(th) / q), np.rint(v * dt * np.sin(th) / q)], 1)
    P0 = np.rint(np.asarray(z0) / q)
    pk = np.zeros(K)
    for g in range(3):
        Gl = np.rint(goals[g].astype(np.float64) / q)
        Q = -np.hypot(*((P0 + S - Gl) * q).T)
        for b in range(9):
            pi = np.exp(float(beta[b]) * (Q - Q.max()))
            pk += belief[g, b] * pi / pi.sum()
    ref = np.zeros(256 * 256)
    for k in range(K):
        p = P0 + S[k]
        ref[int(np.floor(p[1] / 65536)) * 256 + int(np.floor(p[0] / 65536))] += pk[k]
    got = out["counts"][0].reshape(-1).astype(float)
    nz = ref > 0
    assert np.all(got[~nz] == 0)
    z = (got[nz] - N * ref[nz]) / np.sqrt(N * ref[nz] * (1 - ref[nz]))
    assert np.max(np.abs(z)) < 5


def test_counting_invariant_and_trace_consistency(orc):
    sc = scenes.config1()
    h = sc.humans[0]
    belief = scenes.random_belief(h.G, h.B, seed=1)
    grid = (1.0, 1.0, 0.1, 24, 40)  # small grid so that particles leave it
    kw = dict(K=h.K, speed=h.speed, dt=h.dt, beta=h.beta, goals=h.goals, grid=grid, z0=h.start,
              belief=belief, N=3000, H=h.H, seed=0, human=0, cycle=0)
    out = orc.predict(trace=True, **kw)
    assert np.all(out["counts"].reshape(h.H, -1).sum(1) + out["offgrid"] == 3000)
    assert out["offgrid"].max() > 0
    for t in range(h.H):
        cells = out["trace_cell"][:, t]
        hist = np.bincount(cells[cells >= 0], minlength=24 * 40)
        assert np.array_equal(hist, out["counts"][t].reshape(-1))
        assert np.count_nonzero(cells < 0) == out["offgrid"][t]
    # the subset replay reproduces the same particles; thread count does not matter
    idx = np.array([5, 17, 2999, 0])
    sub = orc.predict(trace=True, idx=idx, counts=False, nthreads=1, **kw)
    assert np.array_equal(sub["trace_k"], out["trace_k"][idx])
    assert np.array_equal(sub["trace_pair"], out["trace_pair"][idx])
    one = orc.predict(nthreads=1, **kw)
    assert np.array_equal(one["counts"], out["counts"])


def test_tie_check_classifies(orc):
    sc = scenes.config1()
    h = sc.humans[0]
    belief = scenes.random_belief(h.G, h.B, seed=2)
    kw = dict(K=h.K, speed=h.speed, dt=h.dt, beta=h.beta, goals=h.goals, grid=h.grid,
              z0=h.start, belief=belief, N=200, H=h.H, seed=0, human=0, cycle=0)
    out = orc.predict(trace=True, **kw)
    st, first = orc.tie_check(other_pair=out["trace_pair"], other_k=out["trace_k"], **kw)
    assert np.all(st == 0) and np.all(first == -1)
    bad = out["trace_k"].copy()
    bad[10, 3] = (bad[10, 3] + 3) % h.K
    st, first = orc.tie_check(other_pair=out["trace_pair"], other_k=bad, **kw)
    assert st[10] == 2 and first[10] == 4 and np.count_nonzero(st) == 1
    # an explained change: the window is wide enough to cover the whole CDF
    st, first = orc.tie_check(other_pair=out["trace_pair"], other_k=bad, window=2.0, **kw)
    assert st[10] == 1


def _replay(h, belief, torch_philox, i, H, seed, hid, cyc):
    """Independent replay of particle i (NumPy FP64, PyTorch's Philox): its pair
    j with the pair CDF P and u, and per step the heading k, the normalised CDF
    C / C[-1] and u (Alg. 1 with the documented counters and lattice)."""
    x0, y0, cell, nx, ny = h.grid
    q = cell / 65536
    th = 2 * math.pi * np.arange(h.K) / h.K
    Sx = np.rint(h.speed * h.dt * np.cos(th) / q)
    Sy = np.rint(h.speed * h.dt * np.sin(th) / q)
    P = np.cumsum(belief.reshape(-1))
    up = u_of(torch_philox, seed, i, 0, hid, 2 * cyc, 0)
    j = int(np.argmax(up < P)) if up < P[-1] else int(np.flatnonzero(belief.reshape(-1) > 0)[-1])
    g, b = divmod(j, h.B)
    GX = np.rint((float(h.goals[g][0]) - x0) / q)
    GY = np.rint((float(h.goals[g][1]) - y0) / q)
    X, Y = np.rint((h.start[0] - x0) / q), np.rint((h.start[1] - y0) / q)
    steps = []
    for t in range(1, H + 1):
        d = np.hypot((X + Sx - GX) * q, (Y + Sy - GY) * q)
        C = np.cumsum(np.exp(-float(h.beta[b]) * (d - d.min())))
        u = u_of(torch_philox, seed, i, (t - 1) // 4, hid, 2 * cyc + 1, (t - 1) % 4)
        k = int(np.argmax(u * C[-1] < C)) if u * C[-1] < C[-1] else h.K - 1
        steps.append((k, C / C[-1], u))
        X, Y = X + Sx[k], Y + Sy[k]
    return j, P, up, steps


def test_tie_check_window_boundaries(orc, torch_philox):
    """orc_tie_check, pinned on both sides of every window it applies.  For a
    difference at heading step t the other choice ko must lie across CDF
    boundaries that are all within `window` of u: for ko > k the farthest is
    C[ko-1]/C[-1] - u, for ko < k it is u - C[ko]/C[-1].  For each particle and
    ko in {k-2, k-1, k+1, k+2} that distance is computed here independently;
    the checker must report status 1 (explained) at a window just above it and
    2 at a window just below it, and the first difference at step t; the pair
    draw likewise against pair_window.  An off-by-one boundary, a flipped sign
    or a swapped window fails one side."""
    h = scenes.config1().humans[0]
    belief = scenes.random_belief(h.G, h.B, seed=6)
    N, H, seed, hid, cyc = 48, 6, 3, 4, 2
    kw = dict(K=h.K, speed=h.speed, dt=h.dt, beta=h.beta, goals=h.goals, grid=h.grid,
              z0=h.start, belief=belief, N=N, H=H, seed=seed, human=hid, cycle=cyc)
    out = orc.predict(trace=True, **kw)
    rng = np.random.default_rng(11)
    checked = {1: 0, 2: 0}
    for i in range(N):
        j, P, up, steps = _replay(h, belief, torch_philox, i, H, seed, hid, cyc)
        assert out["trace_pair"][i] == j
        assert [s[0] for s in steps] == list(out["trace_k"][i])
        t = int(rng.integers(1, H + 1))
        k, Cn, u = steps[t - 1]
        for ko in (k - 2, k - 1, k + 1, k + 2):
            if not 0 <= ko < h.K:
                continue
            dist = Cn[ko - 1] - u if ko > k else u - Cn[ko]
            assert dist >= 0
            other = out["trace_k"].copy()
            other[i, t - 1] = ko
            for win, want in ((dist * (1 + 1e-6) + 1e-15, 1), (dist * (1 - 1e-6) - 1e-15, 2)):
                if win < 0:
                    continue
                st, first = orc.tie_check(other_pair=out["trace_pair"][i:i + 1],
                                          other_k=other[i:i + 1], window=win, idx=[i], **kw)
                assert st[0] == want and first[0] == t, (i, t, k, ko, dist, win)
                checked[want] += 1
        # the pair draw: the other implementation picked a neighbouring pair
        for jo in (j - 2, j - 1, j + 1, j + 2):
            if not 0 <= jo < P.size:
                continue
            dist = P[jo - 1] - up if jo > j else up - P[jo]
            other = out["trace_pair"].copy()
            other[i] = jo
            for win, want in ((dist * (1 + 1e-6) + 1e-15, 1), (dist * (1 - 1e-6) - 1e-15, 2)):
                if win < 0:
                    continue
                st, first = orc.tie_check(other_pair=other[i:i + 1],
                                          other_k=out["trace_k"][i:i + 1], pair_window=win,
                                          window=1.0, idx=[i], **kw)
                assert st[0] == want and first[0] == 0, (i, j, jo, dist, win)
    assert checked[1] > 50 and checked[2] > 50
    # the target's 1e-6 window itself: distances found above straddle it
    near = []
    for i in range(N):
        _, _, _, steps = _replay(h, belief, torch_philox, i, H, seed, hid, cyc)
        for t, (k, Cn, u) in enumerate(steps, 1):
            if k + 1 < h.K:
                near.append((Cn[k] - u, i, t, k + 1))
    # an unexplained change stays unexplained at the target window unless its
    # boundary really is within 1e-6 of u
    for dist, i, t, ko in sorted(near)[:5] + sorted(near)[-3:]:
        other = out["trace_k"].copy()
        other[i, t - 1] = ko
        st, _ = orc.tie_check(other_pair=out["trace_pair"][i:i + 1], other_k=other[i:i + 1],
                              window=1e-6, idx=[i], **kw)
        assert st[0] == (1 if dist <= 1e-6 else 2)
