"""Seeded synthetic scenes (input generator shared by tests and the benchmark).

This module holds no arithmetic of the prediction method: it only draws scene
geometry, model grids and sizes with ``numpy.random.Generator(PCG64(1000+c))``.
Observed tracks are produced afterwards by a track simulator (the oracle's in
the tests, the library's in the benchmark), both of which follow the Boltzmann
policy with a per-human true (beta, goal).

The paper measures on no dataset (it needs none, Sec. II); its real-world
recordings are not released.  The five workloads below are synthetic stand-ins
sized like the paper's runs (Tab. 1: 8192 particles, 10 goals, 5 beta values,
96 controls; Sec. IV-B: 5 humans, 21 goals, 418x195 grid at 5 cm) and scaled up
to the many-human serving regime.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

BETA_4 = np.array([0.1, 1.0, 10.0, 100.0], np.float32)
BETA_9 = (10.0 ** (-2.0 + 0.5 * np.arange(9))).astype(np.float32)


@dataclasses.dataclass
class Human:
    hid: int                      # stable human id (keys the random streams)
    K: int                        # headings
    speed: float                  # m/s
    dt: float                     # s per step
    beta: np.ndarray              # float32 [B] rationality grid
    goals: np.ndarray             # float32 [G, 2] metres
    grid: Tuple[float, float, float, int, int]   # (x0, y0, cell, nx, ny)
    N: int                        # particles
    H: int                        # prediction horizon (steps)
    start: Tuple[float, float]    # metres, first observed position
    true_beta: float              # simulator's rationality
    true_goal: int                # simulator's goal index
    n_obs: int                    # observed transitions before the first prediction

    @property
    def B(self) -> int:
        return int(self.beta.size)

    @property
    def G(self) -> int:
        return int(self.goals.shape[0])

    @property
    def frame(self):
        return self.grid[:3]


@dataclasses.dataclass
class Scene:
    name: str
    humans: List[Human]
    seed: int = 0                 # Philox seed for particles and simulated tracks

    @property
    def particle_steps(self) -> int:
        return int(sum(h.N * h.H for h in self.humans))


def _rng(index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 + index))


def config1() -> Scene:
    """1 human, 2 goals in a 6.4 m arena, beta {0.1,1,10,100}, K=8, v=1 m/s,
    dt=0.1 s, 10 observed steps from beta=1 toward goal 0, N=4096, H=20,
    64x64 grid at 0.1 m."""
    r = _rng(1)
    goals = r.uniform(0.0, 6.4, size=(2, 2)).astype(np.float32)
    start = tuple(r.uniform(1.6, 4.8, size=2).tolist())
    h = Human(0, 8, 1.0, 0.1, BETA_4.copy(), goals, (0.0, 0.0, 0.1, 64, 64), 4096, 20,
              start, 1.0, 0, 10)
    return Scene("config1", [h])


def config2() -> Scene:
    """1 human, 3 goals in 12.8 m, 9 beta 1e-2..1e2, K=16, v=1.2, dt=0.05,
    30 observed steps from beta=2 toward goal 0, N=2^18, H=50, 256x256 at 0.05 m."""
    r = _rng(2)
    goals = r.uniform(0.0, 12.8, size=(3, 2)).astype(np.float32)
    start = tuple(r.uniform(3.2, 9.6, size=2).tolist())
    h = Human(0, 16, 1.2, 0.05, BETA_9.copy(), goals, (0.0, 0.0, 0.05, 256, 256), 1 << 18, 50,
              start, 2.0, 0, 30)
    return Scene("config2", [h])


def config3(n_humans: int = 16, n_obs: int = 20) -> Scene:
    """16 humans, N_h = round(2^U(14,18)), G_h ~ U{2..6} goals in 12.8 m,
    9 beta, K=16, v=1.2, dt=0.02, H=100, 256x256 at 0.05 m each; true beta
    log-uniform in [0.1, 50] and a true goal per human."""
    r = _rng(3)
    humans = []
    for h in range(n_humans):
        N = int(round(2.0 ** r.uniform(14.0, 18.0)))
        G = int(r.integers(2, 7))
        goals = r.uniform(0.0, 12.8, size=(G, 2)).astype(np.float32)
        start = tuple(r.uniform(3.2, 9.6, size=2).tolist())
        tb = float(math.exp(r.uniform(math.log(0.1), math.log(50.0))))
        tg = int(r.integers(0, G))
        humans.append(Human(h, 16, 1.2, 0.02, BETA_9.copy(), goals,
                            (0.0, 0.0, 0.05, 256, 256), N, 100, start, tb, tg, n_obs))
    return Scene("config3", humans)


@dataclasses.dataclass
class Visit:
    """One human's stay in a continuous-batching run."""
    hid: int                      # fresh stable id of this visit (keys its random streams)
    human: Human                  # identity: N, goals, start, true beta and goal
    arrive: int                   # cycle at which the request is submitted
    depart: int                   # first cycle without it


def config3_churn(n_cycles: int = 10000, n_identities: int = 48, mean_dwell: int = 800,
                  seed: int = 33) -> List[Visit]:
    """Arrivals and departures for the 16-human serving workload: the 16 humans
    of config3 are present at cycle 0; later visitors arrive as a Poisson
    process of rate 16 / mean_dwell per cycle (so that about 16 are present on
    average), with identities drawn uniformly from config3(n_identities) (the
    first 16 are config3's humans); every stay lasts U[mean_dwell / 4,
    7 mean_dwell / 4] cycles.  Visit ids are 1000 + visit index."""
    ids = config3(n_identities).humans
    r = np.random.Generator(np.random.PCG64(seed))
    lo, hi = max(1, mean_dwell // 4), max(2, 7 * mean_dwell // 4)
    visits = []
    for h in ids[:16]:
        visits.append(Visit(1000 + len(visits), h, 0, int(r.integers(lo, hi + 1))))
    rate = 16.0 / mean_dwell
    t = float(r.exponential(1.0 / rate))
    while t < n_cycles:
        c = int(t)
        h = ids[int(r.integers(0, n_identities))]
        visits.append(Visit(1000 + len(visits), h, c, c + int(r.integers(lo, hi + 1))))
        t += float(r.exponential(1.0 / rate))
    return visits


def config5(n_humans: int = 64, n_obs: int = 20) -> Scene:
    """64 humans x N=2^20, 6 goals each, 9 beta, K=32, v=1.2, dt=0.01, H=200,
    512x512 grids at 0.02 m (arena = grid = 10.24 m)."""
    r = _rng(5)
    humans = []
    for h in range(n_humans):
        goals = r.uniform(0.0, 10.24, size=(6, 2)).astype(np.float32)
        start = tuple(r.uniform(2.56, 7.68, size=2).tolist())
        tb = float(math.exp(r.uniform(math.log(0.1), math.log(50.0))))
        tg = int(r.integers(0, 6))
        humans.append(Human(h, 32, 1.2, 0.01, BETA_9.copy(), goals,
                            (0.0, 0.0, 0.02, 512, 512), 1 << 20, 200, start, tb, tg, n_obs))
    return Scene("config5", humans)


@dataclasses.dataclass
class TrackSet:
    """Inputs of the differentiable log-likelihood workload."""
    K: int
    speed: float
    dt: float
    frame: Tuple[float, float, float]
    goals: np.ndarray            # float32 [G, 2] true goals
    starts: np.ndarray           # float64 [N, 2]
    true_beta: np.ndarray        # float32 [N]
    true_goal: np.ndarray        # int64 [N]
    T: int                       # transitions per track
    beta_grid: np.ndarray        # float32 [B] shared log-beta grid (as beta values)


def config4(n_tracks: int = 1024, T: int = 200) -> TrackSet:
    """1024 tracks of 200 transitions (dt=0.05, K=32, v=1.2) from per-track beta
    log-uniform in [0.1, 50] and one of 8 goals uniform in a 12.8 m arena."""
    r = _rng(4)
    goals = r.uniform(0.0, 12.8, size=(8, 2)).astype(np.float32)
    starts = r.uniform(0.0, 12.8, size=(n_tracks, 2))
    tb = np.exp(r.uniform(math.log(0.1), math.log(50.0), size=n_tracks)).astype(np.float32)
    tg = r.integers(0, 8, size=n_tracks)
    return TrackSet(32, 1.2, 0.05, (0.0, 0.0, 0.05), goals, starts, tb, tg, T, BETA_9.copy())


def random_belief(G: int, B: int, seed: int, sparsity: float = 0.0) -> np.ndarray:
    """Seeded Dirichlet(1) belief over [G][B] pairs, optionally with zeroed entries."""
    r = np.random.Generator(np.random.PCG64(seed))
    b = r.gamma(1.0, size=(G, B))
    if sparsity > 0.0:
        mask = r.uniform(size=(G, B)) < sparsity
        mask.flat[int(r.integers(0, G * B))] = False
        b[mask] = 0.0
    return b / b.sum()
