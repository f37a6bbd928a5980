"""The allocation-free log-likelihood adjoint (cap_loglik_backward_noalloc),
called through the C-ABI: its gradients equal cap_loglik_backward's (same
kernels, same fixed summation order: bit for bit) on two calls in a row, the
second smaller than the first (the static scratch keeps the first call's
partial sums), with shared and per-track beta; sizes beyond the scratch are
refused before any launch."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_01122_amd import capred
    return capred


def _inputs(N, T, G, B, per_track, seed, K=16, v=1.2, dt=0.05):
    r = np.random.default_rng(seed)
    th = 2 * np.pi * r.integers(0, K, (N, T)) / K
    steps = v * dt * np.stack([np.cos(th), np.sin(th)], -1)
    start = r.uniform(2, 10, (N, 1, 2))
    tracks = np.concatenate([start, start + np.cumsum(steps, 1)], 1).astype(np.float32)
    lengths = r.integers(0, T + 1, N).astype(np.int32)
    lengths[0] = T
    goals = r.uniform(0, 12.8, (G, 2)).astype(np.float32)
    lb_shape = (N, B) if per_track else (B,)
    log_beta = np.log(np.exp(r.uniform(np.log(0.1), np.log(50), lb_shape))).astype(np.float32)
    dLL = r.standard_normal((N, B, G))
    t = lambda a: torch.tensor(a, device="cuda")
    return K, v, dt, t(tracks), t(lengths), t(goals), t(log_beta), t(dLL)


def test_noalloc_matches_workspace_entry_point(cap):
    cases = [dict(N=300, T=40, G=8, B=9, per_track=False, seed=1),
             dict(N=57, T=23, G=3, B=4, per_track=True, seed=2)]
    for c in cases:
        print(f"[case] noalloc adjoint {c}", flush=True)
        K, v, dt, tracks, lengths, goals, log_beta, dLL = _inputs(**c)
        dg_ref, db_ref = cap.loglik_backward(K, v, dt, tracks, lengths, goals, log_beta, dLL)
        dg = torch.full_like(dg_ref, float("nan"))
        db = torch.full_like(db_ref, float("nan"))
        cap.loglik_backward_noalloc(K, v, dt, tracks, lengths, goals, log_beta, dLL, dg, db)
        torch.cuda.synchronize()
        assert torch.equal(dg, dg_ref), c
        assert torch.equal(db, db_ref), c


def test_noalloc_refuses_sizes_beyond_the_scratch(cap):
    K, v, dt, tracks, lengths, goals, log_beta, dLL = _inputs(8, 3, 2, 2, False, 3)
    N, G, B = 48000, 1, 9        # 48000 * 1 * 11 * 8 B > 4 MiB
    assert cap._lib.cap_loglik_backward_workspace(N, G, B, 0) > 4 << 20
    big = torch.zeros((N, 4, 2), dtype=torch.float32, device="cuda")
    lens = torch.zeros(N, dtype=torch.int32, device="cuda")
    g = torch.zeros((G, 2), dtype=torch.float32, device="cuda")
    lb = torch.zeros(B, dtype=torch.float32, device="cuda")
    d = torch.zeros((N, B, G), dtype=torch.float64, device="cuda")
    dg = torch.zeros((G, 2), dtype=torch.float64, device="cuda")
    db = torch.zeros(B, dtype=torch.float64, device="cuda")
    with pytest.raises(cap.CapError, match="SCRATCH") as e:
        cap.loglik_backward_noalloc(K, v, dt, big, lens, g, lb, d, dg, db)
    assert e.value.status == -5           # CAP_E_CAPACITY
