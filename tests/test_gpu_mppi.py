"""GPU parity of the MPPI consumer (Sec. III-C) against the FP64 oracle, on
predicted grids that the library produced (union of several humans).

FP64 on both sides; the robot state differs only by the last-bit differences
of the two cos/sin implementations, so costs agree to 1e-9 relative for every
sample that never read the grid within 1e-9 m of a cell edge (the oracle flags
those; none occur in these scenes), and the updated controls to 1e-9.
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


def predicted_union(cap, humans, N, H):
    probs = []
    for h in humans:
        bel = torch.tensor(scenes.random_belief(h.G, h.B, seed=h.hid).reshape(h.G, h.B),
                           dtype=torch.float64, device="cuda")
        out = cap.predict_occupancy(cap.model_of(h), h.grid, h.start, bel, N, H, seed=0,
                                    human_id=h.hid)
        probs.append(cap.normalize(out["counts"], N))
    return cap.union_max(probs)


@pytest.mark.parametrize("N,T,tau", [(4096, 40, 5.0), (1000, 25, 50.0), (1, 10, 1.0)])
def test_mppi_step_matches_oracle(orc, cap, N, T, tau):
    humans = scenes.config3().humans[:3]
    note(f"mppi N={N} T={T} tau={tau} on the union of 3 predicted humans")
    occ = predicted_union(cap, humans, 20000, 60)
    torch.cuda.synchronize()
    grid = humans[0].grid
    r = np.random.default_rng(N + T)
    h0 = humans[0]
    z0 = np.array([h0.start[0] - 2.0, h0.start[1] - 1.5, 0.8, 0.6])
    goal = np.array([h0.start[0] + 2.5, h0.start[1] + 2.0, 0.0, 0.0])
    U0 = np.tile([0.0, 0.0], (T, 1)) + r.normal(scale=0.1, size=(T, 2))
    delta = r.normal(scale=[0.8, 0.6], size=(T, N, 2))
    kw = dict(dt=0.1, tau=tau, c_time=0.1, **cap.PAPER_MPPI_COST)
    U = torch.tensor(U0, device="cuda")
    S = cap.mppi_step(z0, goal, U, torch.tensor(delta, device="cuda"), occ=occ, grid=grid, **kw)
    torch.cuda.synchronize()
    S_o, U_o, near = orc.mppi(z0=z0, goal=goal, U=U0, delta=delta, occ=occ.cpu().numpy(),
                              grid=grid, **kw)
    assert np.all(near == 0)
    S = S.cpu().numpy()
    assert np.all(np.abs(S - S_o) <= 1e-9 * np.maximum(1.0, np.abs(S_o)))
    assert np.max(np.abs(U.cpu().numpy() - U_o)) <= 1e-9
    if N > 1:
        assert np.any(S_o >= 1000.0)     # the predictions do enter the cost


def test_mppi_receding_horizon(orc, cap):
    """Five replanning steps, each executing the first control and shifting."""
    humans = scenes.config3().humans[3:5]
    occ = predicted_union(cap, humans, 20000, 50)
    torch.cuda.synchronize()
    occ_h = occ.cpu().numpy()
    grid = humans[0].grid
    T, N, dt = 30, 2048, 0.1
    r = np.random.default_rng(7)
    z = np.array([humans[0].start[0] - 1.5, humans[0].start[1], 0.5, 0.0])
    goal = np.array([humans[0].start[0] + 3.0, humans[0].start[1] + 0.5, 0.0, 0.0])
    U_g = torch.zeros((T, 2), dtype=torch.float64, device="cuda")
    U_o = np.zeros((T, 2))
    kw = dict(dt=dt, tau=10.0, **cap.PAPER_MPPI_COST)
    note("mppi receding horizon, 5 steps")
    for k in range(5):
        delta = r.normal(scale=[0.8, 0.6], size=(T, N, 2))
        cap.mppi_step(z, goal, U_g, torch.tensor(delta, device="cuda"), occ=occ, grid=grid, **kw)
        _, U_o, near = orc.mppi(z0=z, goal=goal, U=U_o, delta=delta, occ=occ_h, grid=grid, **kw)
        assert np.all(near == 0)
        Ug = U_g.cpu().numpy()
        assert np.max(np.abs(Ug - U_o)) <= 1e-9, k
        # execute the first control (oracle's) and shift the references
        a, w = U_o[0]
        z = np.array([z[0] + z[2] * np.cos(z[3]) * dt, z[1] + z[2] * np.sin(z[3]) * dt,
                      z[2] + a * dt, z[3] + w * dt])
        U_o = np.vstack([U_o[1:], U_o[-1:]])
        U_g = torch.tensor(U_o, device="cuda")
