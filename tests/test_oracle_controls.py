"""Pins of the oracle's multi-speed control set (speeds x headings, u = s K + k;
the 96-control experiments of Sec. IV) and of the speed mask that removes fast
controls of a stationary human (Q = -inf, Sec. IV-B).

* lattice steps of two speeds in closed form; one speed given as a list is the
  single-speed oracle bit for bit;
* beta -> 0: the control is uniform over the allowed ones, exactly the
  floor(u n_allowed)-th allowed control for PyTorch's Philox u;
* beta -> inf: particles follow the brute-force greedy path over the allowed
  controls (masked controls never appear);
* exact enumeration over all U^H control paths and pairs (with and without a
  mask) against 400k-particle Monte Carlo;
* control recovery inverts the simulator's lattice steps; the nearest control
  found by brute force over all U controls equals it;
* Bayes: the posterior equals the direct product of the U-control policy.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.stats


def u_of(torch_philox, seed, c0, c1, c2, c3, word):
    w = torch_philox(seed, c0, c1, c2, c3)[word]
    return ((int(w) >> 9) * 2 + 1) * 2.0 ** -24


def steps_table(K, speeds, dt, q):
    th = 2 * np.pi * np.arange(K) / K
    return np.concatenate([np.stack([np.rint(v * dt * np.cos(th) / q),
                                     np.rint(v * dt * np.sin(th) / q)], 1) for v in speeds])


def allowed_of(K, S, mask):
    m = mask or (1 << S) - 1
    return np.repeat([(m >> s) & 1 == 1 for s in range(S)], K)


def test_lattice_steps_two_speeds(orc):
    Sx, Sy = orc.lattice_steps(4, 0.0, 0.1, 0.1, speeds=[0.5, 1.0])
    assert list(Sx) == [32768, 0, -32768, 0, 65536, 0, -65536, 0]
    assert list(Sy) == [0, 32768, 0, -32768, 0, 65536, 0, -65536]
    with pytest.raises(ValueError):
        orc.lattice_steps(4, 0.0, 0.1, 0.1, speeds=[0.5, -1.0])
    with pytest.raises(ValueError):
        orc.lattice_steps(16, 0.0, 0.1, 0.1, speeds=[0.1] * 9)   # more than 8 speeds


def test_one_speed_list_is_single_speed(orc):
    kw = dict(K=8, dt=0.1, beta=np.array([0.5, 4.0], np.float32),
              goals=np.array([[1.1, 5.2], [4.9, 0.7]], np.float32), grid=(0, 0, 0.1, 64, 64),
              z0=(3.1, 2.9), belief=np.array([0.2, 0.3, 0.1, 0.4]), N=3000, H=12, seed=5,
              trace=True)
    a = orc.predict(speed=1.1, **kw)
    b = orc.predict(speed=0.0, speeds=[1.1], **kw)
    for key in ("counts", "offgrid", "trace_k", "trace_pair"):
        assert np.array_equal(a[key], b[key])


@pytest.mark.parametrize("mask", [0, 0b011, 0b100])
def test_beta_to_zero_uniform_over_allowed(orc, torch_philox, mask):
    K, speeds = 8, [0.4, 0.8, 1.2]
    allowed = np.nonzero(allowed_of(K, 3, mask))[0]
    N, H = 400, 6
    out = orc.predict(K=K, speed=0.0, speeds=speeds, speed_mask=mask, dt=0.1,
                      beta=np.array([1e-12], np.float32), goals=np.array([[5, 5]], np.float32),
                      grid=(0, 0, 0.1, 64, 64), z0=(3.2, 3.2), belief=np.ones(1), N=N, H=H,
                      seed=1, human=4, cycle=3, trace=True)
    for i in range(0, N, 5):
        for t in range(1, H + 1):
            u = u_of(torch_philox, 1, i, (t - 1) // 4, 4, 7, (t - 1) % 4)
            assert out["trace_k"][i, t - 1] == allowed[math.floor(u * allowed.size)], (i, t)


@pytest.mark.parametrize("mask", [0, 0b001])
def test_beta_to_inf_greedy_over_allowed(orc, mask):
    K, speeds, dt, cell = 8, [0.3, 0.9, 1.5], 0.1, 0.1
    goals = np.array([[5.13, 1.37], [0.71, 4.46]], np.float32)
    z0 = (3.03, 2.91)
    N, H = 1000, 30
    out = orc.predict(K=K, speed=0.0, speeds=speeds, speed_mask=mask, dt=dt,
                      beta=np.array([1e6], np.float32), goals=goals, grid=(0, 0, cell, 64, 64),
                      z0=z0, belief=np.array([0.4, 0.6]), N=N, H=H, seed=4, trace=True)
    q = cell / 65536
    S = steps_table(K, speeds, dt, q)
    ok = allowed_of(K, 3, mask)
    P0 = np.rint(np.array(z0) / q)
    for g in range(2):
        Gl = np.rint(goals[g].astype(np.float64) / q)
        p = P0.copy()
        path = []
        for t in range(H):
            dist = np.where(ok, np.hypot(*((p + S - Gl) * q).T), np.inf)
            u = int(np.argmin(dist))
            assert np.sort(dist)[1] - dist[u] > 1e-9
            p = p + S[u]
            path.append(u)
        sel = out["trace_pair"] == g
        assert sel.sum() > 0
        assert np.all(out["trace_k"][sel] == np.array(path, np.uint8)[None])
    assert np.all(ok[out["trace_k"]])


def _exact(K, speeds, mask, dt, cell, beta, goals, belief, z0, H, nx, ny):
    q = cell / 65536
    S = steps_table(K, speeds, dt, q)
    ok = allowed_of(K, len(speeds), mask)
    P0 = np.rint(np.asarray(z0, np.float64) / q)
    dist = np.zeros((H, ny * nx + 1))
    B = beta.size
    for g in range(goals.shape[0]):
        Gl = np.rint(goals[g].astype(np.float64) / q)
        for b in range(B):
            pb = belief[g * B + b]
            for path in itertools.product(np.nonzero(ok)[0], repeat=H):
                p, prob, cells = P0.copy(), pb, []
                for u in path:
                    Q = -np.hypot(*((p + S - Gl) * q).T)
                    w = np.where(ok, np.exp(float(beta[b]) * (Q - Q[ok].max())), 0.0)
                    prob *= w[u] / w.sum()
                    p = p + S[u]
                    cx, cy = int(np.floor(p[0] / 65536)), int(np.floor(p[1] / 65536))
                    cells.append(cy * nx + cx if (0 <= cx < nx and 0 <= cy < ny) else ny * nx)
                for t, c in enumerate(cells):
                    dist[t, c] += prob
    return dist


@pytest.mark.parametrize("mask", [0, 0b01])
def test_enumeration_matches_monte_carlo_two_speeds(orc, mask):
    K, speeds, dt, cell, nx, ny, H = 4, [0.5, 1.0], 0.1, 0.05, 16, 16, 3
    beta = np.array([0.5, 8.0], np.float32)
    goals = np.array([[0.61, 0.13], [0.09, 0.47]], np.float32)
    belief = np.array([0.1, 0.3, 0.25, 0.35])
    z0 = (0.4137, 0.3862)
    exact = _exact(K, speeds, mask, dt, cell, beta, goals, belief, z0, H, nx, ny)
    assert np.allclose(exact.sum(1), 1.0)
    N = 400000
    out = orc.predict(K=K, speed=0.0, speeds=speeds, speed_mask=mask, dt=dt, beta=beta,
                      goals=goals, grid=(0, 0, cell, nx, ny), z0=z0, belief=belief, N=N, H=H,
                      seed=23)
    for t in range(H):
        mc = np.concatenate([out["counts"][t].reshape(-1), [out["offgrid"][t]]]).astype(float)
        e = exact[t] * N
        assert np.all(mc[e == 0] == 0)
        keep = e >= 5
        obs = np.append(mc[keep], mc[~keep].sum())
        exp_ = np.append(e[keep], e[~keep].sum())
        if exp_[-1] < 5:
            obs[-2] += obs[-1]
            exp_[-2] += exp_[-1]
            obs, exp_ = obs[:-1], exp_[:-1]
        p = scipy.stats.chisquare(obs, exp_ * obs.sum() / exp_.sum()).pvalue
        assert p > 1e-4, (t, p)


def test_recover_controls_two_speeds(orc):
    K, speeds, dt, cell = 16, [0.25, 0.75, 1.5], 0.05, 0.05
    frame = (0.0, 0.0, cell)
    lat, pos = orc.simulate_tracks(K=K, speed=0.0, speeds=speeds, dt=dt, frame=frame,
                                   start=np.array([[6.0, 6.0], [3.0, 9.0]]), beta=[0.8, 6.0],
                                   goal=np.array([[9.0, 2.0], [1.0, 1.0]]), T=300, seed=2)
    Sx, Sy = orc.lattice_steps(K, 0.0, dt, cell, speeds=speeds)
    th = 2 * np.pi * np.arange(K) / K
    cont = np.concatenate([np.stack([v * dt * np.cos(th), v * dt * np.sin(th)], 1)
                           for v in speeds])
    seen = set()
    for n in range(2):
        dl = np.diff(lat[n], axis=0)
        truth = [int(np.nonzero((Sx == d[0]) & (Sy == d[1]))[0][0]) for d in dl]
        us, _ = orc.recover_controls(K, pos[n], speed=0.0, dt=dt, speeds=speeds)
        assert list(us) == truth
        d = np.diff(pos[n].astype(np.float64), axis=0)
        near = np.argmin(np.hypot(d[:, None, 0] - cont[None, :, 0],
                                  d[:, None, 1] - cont[None, :, 1]), axis=1)
        assert list(near) == truth
        seen |= {u // K for u in truth}
    assert len(seen) >= 2          # the tracks use more than one speed


def test_bayes_direct_product_two_speeds(orc):
    K, speeds, dt = 8, [0.4, 1.2], 0.1
    goals = np.array([[5.0, 1.0], [1.0, 5.0], [4.0, 4.5]], np.float32)
    beta = np.array([0.1, 0.7, 2.0], np.float32)
    _, obs = orc.simulate_tracks(K=K, speed=0.0, speeds=speeds, dt=dt, frame=(0, 0, 0.1),
                                 start=np.array([[2.0, 2.0]]), beta=[1.5], goal=goals[:1],
                                 T=12, seed=3)
    obs = obs[0]
    lb, b, _ = orc.belief_update(K=K, speed=0.0, speeds=speeds, dt=dt, beta=beta, goals=goals,
                                 obs=obs)
    th = 2 * np.pi * np.arange(K) / K
    s = np.concatenate([np.stack([(v * dt * np.cos(th)).astype(np.float32),
                                  (v * dt * np.sin(th)).astype(np.float32)], 1)
                        for v in speeds]).astype(np.float64)
    exact_steps = np.concatenate([np.stack([v * dt * np.cos(th), v * dt * np.sin(th)], 1)
                                  for v in speeds])
    prod = np.full((3, 3), 1.0 / 9)
    for t in range(obs.shape[0] - 1):
        d = obs[t + 1].astype(np.float64) - obs[t]
        u = int(np.argmin(np.hypot(d[0] - exact_steps[:, 0], d[1] - exact_steps[:, 1])))
        z = obs[t].astype(np.float64)
        for g in range(3):
            Q = -np.hypot(z[0] + s[:, 0] - goals[g, 0], z[1] + s[:, 1] - goals[g, 1])
            for j, bt in enumerate(beta.astype(np.float64)):
                e = np.exp(bt * Q)
                prod[g, j] *= e[u] / e.sum()
    prod /= prod.sum()
    assert np.allclose(b, prod, rtol=1e-10, atol=0)


def test_tie_check_rejects_masked_control(orc):
    kw = dict(K=4, speed=0.0, speeds=[0.5, 1.0], speed_mask=0b01, dt=0.1,
              beta=np.array([1.0], np.float32), goals=np.array([[3, 3]], np.float32),
              grid=(0, 0, 0.1, 64, 64), z0=(1.0, 1.0), belief=np.ones(1), N=50, H=3, seed=0)
    ref = orc.predict(trace=True, **kw)
    st, _ = orc.tie_check(other_pair=ref["trace_pair"], other_k=ref["trace_k"], **kw)
    assert np.all(st == 0)
    bad = ref["trace_k"].copy()
    bad[:, 0] += 4                      # the same heading at the masked speed
    st, first = orc.tie_check(other_pair=ref["trace_pair"], other_k=bad, **kw)
    assert np.all(st == 2) and np.all(first == 1)
