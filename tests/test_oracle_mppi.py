"""Pins of the oracle's MPPI consumer (Sec. III-C, local planner):

* no perturbation: the references are unchanged and the straight-line cost
  equals its closed form (arithmetic sums);
* constant turn rate: the Euler positions follow the geometric-series closed
  form of sum_s exp(i s omega dt);
* one sample: the update is that sample's perturbation;
* tau -> infinity: the update is the plain mean of the perturbations (NumPy);
  tau -> 0: the perturbation of the cheapest sample;
* a constant time cost shifts every S equally and leaves the update unchanged;
* the collision term adds exactly w_coll for each step spent in a cell whose
  predicted probability reaches the threshold, and nothing below it.
"""
import numpy as np
import pytest


def test_straight_line_closed_form(orc):
    T, dt, v0 = 12, 0.25, 0.8
    g = np.array([4.0, 0.5, 0.3, 0.0])
    S, U, _ = orc.mppi(z0=[0, 0, v0, 0], goal=g, U=np.zeros((T, 2)), delta=np.zeros((T, 3, 2)),
                       dt=dt, tau=1.0, Q=(3, 3, 10, 0), Qf=(0.6, 0.6, 2, 0), R=(2, 1),
                       c_time=0.05)
    assert np.array_equal(U, np.zeros((T, 2)))
    a, n = v0 * dt, T - 1
    st1, st2 = n * (n + 1) / 2, n * (n + 1) * (2 * n + 1) / 6
    run = 3 * (a * a * st2 - 2 * a * g[0] * st1 + n * g[0] ** 2) + n * (3 * g[1] ** 2 +
                                                                        10 * (v0 - g[2]) ** 2 + 0.05)
    term = 0.6 * (a * T - g[0]) ** 2 + 0.6 * g[1] ** 2 + 2 * (v0 - g[2]) ** 2
    assert np.allclose(S, run + term, rtol=1e-13, atol=0)


def test_constant_turn_geometric_series(orc):
    T, dt, v0, w, th0 = 30, 0.1, 1.3, 0.7, 0.4
    gx = 2.0
    S, _, _ = orc.mppi(z0=[0, 0, v0, th0], goal=[gx, 0, 0, 0], U=np.tile([0.0, w], (T, 1)),
                       delta=np.zeros((T, 1, 2)), dt=dt, tau=1.0, Q=(1, 0, 0, 0),
                       Qf=(0, 0, 0, 0), R=(0, 0))
    t = np.arange(1, T)
    q = np.exp(1j * w * dt)
    z = v0 * dt * np.exp(1j * th0) * (1 - q ** t) / (1 - q)   # sum_{s<t} of the step
    assert np.isclose(S[0], np.sum((z.real - gx) ** 2), rtol=1e-12)


def test_update_limits(orc):
    r = np.random.default_rng(5)
    T, N = 8, 64
    U0 = r.normal(size=(T, 2))
    d = r.normal(size=(T, N, 2))
    kw = dict(z0=[1, 2, 0.5, 0.3], goal=[3, 3, 0, 0], U=U0, dt=0.2, Q=(3, 3, 10, 0),
              Qf=(0.6, 0.6, 2, 0), R=(2, 1))
    _, U1, _ = orc.mppi(delta=d[:, :1], tau=1.0, **kw)
    assert np.allclose(U1, U0 + d[:, 0], rtol=0, atol=1e-15)
    _, Uinf, _ = orc.mppi(delta=d, tau=1e15, **kw)
    assert np.allclose(Uinf, U0 + d.mean(axis=1), rtol=0, atol=1e-12)
    S, U0t, _ = orc.mppi(delta=d, tau=1e-9, **kw)
    assert np.array_equal(U0t, U0 + d[:, int(np.argmin(S))])
    S2, Uc, _ = orc.mppi(delta=d, tau=0.7, c_time=3.5, **kw)
    S1, Ub, _ = orc.mppi(delta=d, tau=0.7, **kw)
    assert np.allclose(S2 - S1, 3.5 * (T - 1), rtol=0, atol=1e-9)
    assert np.allclose(Uc, Ub, rtol=0, atol=1e-12)


def test_collision_term(orc):
    T, dt, v0 = 10, 0.5, 0.4       # straight along y = 0.25: x_t = 0.05 + 0.2 t, cells of 0.1 m
    grid = (0.0, 0.0, 0.1, 40, 10)
    occ = np.zeros((12, 10, 40), np.float32)
    occ[2, 2, 6] = 0.5             # step 3: x = 0.65 -> cell 6
    occ[4, 2, 10] = 0.1            # step 5: x = 1.05 -> cell 10, at the threshold
    occ[6, 2, 14] = 0.0999         # step 7: x = 1.45 -> cell 14, below the threshold
    occ[8, 2, 19] = 0.9            # step 9: x = 1.85 -> cell 18, a neighbour: no hit
    occ[9, 2, 20] = 0.9            # step 10 = T: terminal step carries no collision cost
    kw = dict(z0=[0.05, 0.25, v0, 0.0], goal=[5, 0.25, v0, 0], U=np.zeros((T, 2)),
              delta=np.zeros((T, 2, 2)), dt=dt, tau=1.0, Q=(3, 3, 10, 0), Qf=(0.6, 0.6, 2, 0),
              R=(2, 1))
    S0, _, _ = orc.mppi(**kw)
    S1, _, near = orc.mppi(occ=occ, grid=grid, w_coll=1000.0, p_coll=0.1, **kw)
    assert np.allclose(S1 - S0, 2000.0, rtol=0, atol=1e-9)
    assert np.all(near == 0)
