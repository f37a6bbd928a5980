"""GPU parity of the Gaussian-smoothed occupancy and the multi-human union
against the oracle (direct 2-D FP64 sum; element-wise maximum).

Smoothing tolerance, derived from the FP32 arithmetic: every term is
non-negative, the weights are FP32 roundings of the normalised 1-D kernel
(relative 2^-24 each), each pass accumulates 2r+1 products with FMAs (at most
2r+1 roundings), and the final division rounds once, so the relative error of
an output is at most (4r + 6) 2^-24 of the exact value.
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


def check_smooth(orc, cap, counts, N, sigma, radius):
    note(f"smooth {counts.shape} N={N} sigma={sigma} r={radius}")
    c = torch.tensor(counts.view(np.int32), device="cuda")
    p = cap.smooth_occupancy(c, N, sigma, radius)
    torch.cuda.synchronize()
    got = p.cpu().numpy().astype(np.float64)
    ref = orc.smooth(counts, N, sigma, radius)
    tol = (4 * radius + 6) * 2.0 ** -24
    assert np.all(np.abs(got - ref) <= tol * ref), np.max(np.abs(got - ref) / np.maximum(ref, 1e-300))
    assert np.array_equal(got == 0, ref == 0)
    return got


@pytest.mark.parametrize("shape,sigma,radius", [((3, 70, 300), 1.0, 3), ((2, 33, 257), 0.6, 1),
                                                ((1, 100, 40), 4.0, 16), ((4, 1, 1), 1.0, 2),
                                                ((2, 5, 2), 2.0, 5), ((3, 64, 64), 1.0, 0)])
def test_smooth_random(orc, cap, shape, sigma, radius):
    r = np.random.default_rng(radius * 7 + shape[1])
    counts = r.integers(0, 3000, shape).astype(np.uint32)
    counts[r.random(shape) < 0.6] = 0          # sparse, like late-step histograms
    N = int(counts.reshape(shape[0], -1).sum(1).max()) + 11
    check_smooth(orc, cap, counts, N, sigma, radius)


def test_smooth_of_prediction(orc, cap):
    h = scenes.config2().humans[0]
    belief = scenes.random_belief(h.G, h.B, seed=9)
    note("predict config2 size, then smooth sigma=1 r=3")
    out = cap.predict_occupancy(cap.model_of(h), h.grid, h.start,
                                torch.tensor(belief.reshape(h.G, h.B), dtype=torch.float64,
                                             device="cuda"), h.N, h.H, seed=0)
    torch.cuda.synchronize()
    counts = out["counts"].cpu().numpy().view(np.uint32)
    got = check_smooth(orc, cap, counts, h.N, 1.0, 3)
    # mass is conserved away from the border: every step's particles lie well inside
    inner = counts[:, :3, :].sum() + counts[:, -3:, :].sum() + counts[:, :, :3].sum() + \
        counts[:, :, -3:].sum()
    if inner == 0:
        mass = got.reshape(h.H, -1).sum(1)
        ongrid = counts.reshape(h.H, -1).sum(1) / h.N
        assert np.allclose(mass, ongrid, rtol=1e-5)


def test_smooth_rejects(cap):
    c = torch.zeros((2, 8, 8), dtype=torch.int32, device="cuda")
    for kw in (dict(sigma=1.0, radius=17), dict(sigma=0.0, radius=2), dict(sigma=1.0, radius=-1)):
        with pytest.raises(cap.CapError):
            cap.smooth_occupancy(c, 10, **kw)
    with pytest.raises(cap.CapError):
        cap.smooth_occupancy(c, 0)


def test_union_max(orc, cap):
    r = np.random.default_rng(11)
    for n_h, shape in [(16, (100, 64, 64)), (1, (3, 5, 7)), (5, (2, 3, 3))]:
        note(f"union of {n_h} grids {shape}")
        gs = [r.random(shape).astype(np.float32) * (r.random(shape) < 0.3) for _ in range(n_h)]
        dev = [torch.tensor(g, device="cuda") for g in gs]
        u = cap.union_max(dev)
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), orc.union_max(gs))
        # in place into the first grid
        cap.union_max(dev, out=dev[0])
        torch.cuda.synchronize()
        assert np.array_equal(dev[0].cpu().numpy(), orc.union_max(gs))
    # misaligned views take the scalar path
    base = torch.tensor(r.random(1001).astype(np.float32), device="cuda")
    a, b = base[1:1001], torch.tensor(r.random(1000).astype(np.float32), device="cuda")
    u = cap.union_max([a, b])
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), orc.union_max([a.cpu().numpy(), b.cpu().numpy()]))
