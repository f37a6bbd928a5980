"""FP64 CPU oracle for confidence-aware particle prediction.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  The product
library never imports, links or calls it, and it shares no code with the HIP
path: its own Philox, lattice tables, control recovery, policy, belief update,
rollout, histograms and log-likelihood, all in ``capred_oracle.c``.

Each function follows a passage of the paper (Lu, Bui, Lyu, Chen, "Fast
Confidence-Aware Human Prediction via Hardware-accelerated Bayesian Inference
for Safe Robot Navigation"):

* ``belief_update``  -- Eq. (beta_update) and its log-space form (Sec. III-B):
  static (beta, g), uniform prior (Sec. III-B), one log-sum-exp per update.
* ``predict``        -- Alg. 1: bootstrapped (beta, g) draw per particle,
  Boltzmann heading draws (Eq. human_softmax_policy) at the particle's own
  state, discretised kinematic step (Eq. human_dynamics), emplacement per step.
* ``recover_controls`` -- control recovery from consecutive states (flatness,
  Sec. III-A).
* ``loglik`` / ``loglik_grad`` -- product form of Eq. (beta_update) over a
  track, and its exact derivative with respect to goals and log beta.
* ``simulate_tracks`` -- synthetic humans following the same Boltzmann policy.
* ``normalize``      -- counts / N (Alg. 1 output p(z) per grid).

Pins (tests/test_oracle_*.py): Philox against PyTorch's Philox4x32-10 engine;
closed-form K=4 policy; beta->0 uniform and beta->inf argmax limits; exact
enumeration of Eq. (human_prediction)/(human_prediction_multi_step) on tiny
inputs; brute-force Bayes by direct products; the counting invariant; central
finite differences for the gradient.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "capred_oracle.c")
_LIB = os.path.join(_HERE, "libcapred_oracle.so")
_lock = threading.Lock()
_lib = None

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no fast-math, no FP contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _nullable(ptype):
    """ndpointer that also accepts None (passed as NULL)."""
    def from_param(cls, obj):
        if obj is None:
            return None
        return ptype.from_param(obj)
    return type(ptype.__name__ + "_or_null", (ptype,), {"from_param": classmethod(from_param)})


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_LIB)
            i64, i32, u32, u64, d = C.c_int64, C.c_int, C.c_uint32, C.c_uint64, C.c_double
            L.orc_philox_bulk.argtypes = [i64, u32, u32, u32, u32, u64, _u32p]
            L.orc_philox_bulk.restype = None
            L.orc_uniform24.argtypes = [u32]
            L.orc_uniform24.restype = d
            L.orc_lattice_steps.argtypes = [i32, i32, _f64p, d, d, _i32p, _i32p]
            L.orc_lattice_steps.restype = i32
            L.orc_predict.argtypes = [
                i32, i32, _f64p, u32, d, i32, _f32p, i32, _f32p, d, d, d, i32, i32, d, d, _f64p,
                i64, i32, u64, u32, u32, _nullable(_i64p), i64,
                _nullable(_u32p), _nullable(_u32p), _nullable(_u8p), _nullable(_i32p),
                _nullable(_i32p), i32]
            L.orc_predict.restype = i32
            L.orc_tie_check.argtypes = [
                i32, i32, _f64p, u32, d, i32, _f32p, i32, _f32p, d, d, d, d, d, _f64p,
                i64, i32, u64, u32, u32, _nullable(_i64p), i64,
                _i32p, _u8p, d, d, _i32p, _i32p, i32]
            L.orc_tie_check.restype = i32
            L.orc_recover_controls.argtypes = [i32, i32, _f64p, d, _f32p, i32, _i32p,
                                               _nullable(_f64p)]
            L.orc_recover_controls.restype = i32
            L.orc_belief_update.argtypes = [i32, i32, _f64p, d, i32, _f32p, i32, _f32p, _f32p, i32,
                                            _f64p, _nullable(_f64p), _nullable(_f64p), i32]
            L.orc_belief_update.restype = i32
            L.orc_loglik.argtypes = [i32, d, d, _f32p, _i32p, i32, i32, _f64p, i32, _f64p, i32,
                                     i32, _f64p, i32]
            L.orc_loglik.restype = i32
            L.orc_loglik_grad.argtypes = [i32, d, d, _f32p, _i32p, i32, i32, _f64p, i32, _f64p,
                                          i32, i32, _f64p, _f64p, _f64p]
            L.orc_loglik_grad.restype = i32
            L.orc_simulate_tracks.argtypes = [i32, i32, _f64p, d, d, d, d, i32, i32, _f64p, _f32p,
                                              _f32p,
                                              u64, u32, _nullable(_i64p), _nullable(_f32p)]
            L.orc_simulate_tracks.restype = i32
            L.orc_smooth.argtypes = [_u32p, i32, i32, i32, i64, d, i32, _nullable(_i64p), i64,
                                     _f64p, i32]
            L.orc_smooth.restype = i32
            L.orc_union_max.argtypes = [C.POINTER(C.POINTER(C.c_float)), i32, i64, _f32p]
            L.orc_union_max.restype = i32
            L.orc_mppi.argtypes = [_f64p, _f64p, i32, d, i32, _f64p, _f64p, _nullable(_f32p), i32,
                                   d, d, d, i32, i32, _f64p, _f64p, _f64p, d, d, d, d, _f64p,
                                   _f64p, _nullable(_i32p)]
            L.orc_mppi.restype = i32
            _lib = L
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def _speeds(speed, speeds):
    """Speeds of the control set (m/s) as FP64: `speeds` if given, else the one `speed`."""
    v = [speed] if speeds is None else list(speeds)
    return np.ascontiguousarray(v, np.float64)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


# --------------------------------------------------------------------------- RNG
def philox_bulk(n: int, c0: int, c1: int, c2: int, c3: int, seed: int) -> np.ndarray:
    """Philox4x32-10 blocks for counters (c0+i, c1, c2, c3), i < n -> uint32 [n, 4]."""
    out = np.empty((n, 4), np.uint32)
    lib().orc_philox_bulk(n, c0 & 0xFFFFFFFF, c1, c2, c3, seed, out)
    return out


def uniform24(words: np.ndarray) -> np.ndarray:
    """u = (2*(w>>9)+1) * 2^-24 in (0,1)."""
    w = np.asarray(words, np.uint64)
    return ((w >> np.uint64(9)).astype(np.float64) * 2.0 + 1.0) * 2.0 ** -24


def lattice_steps(K: int, speed: float, dt: float, cell: float, speeds=None):
    """Lattice steps of the U = S*K controls, u = s*K + k."""
    v = _speeds(speed, speeds)
    Sx = np.empty(K * v.size, np.int32)
    Sy = np.empty(K * v.size, np.int32)
    _check(lib().orc_lattice_steps(K, v.size, v, dt, cell, Sx, Sy), "lattice_steps")
    return Sx, Sy


# ------------------------------------------------------------------ prediction
def predict(*, K, speed, dt, beta, goals, grid, z0, belief, N, H, seed=0, human=0, cycle=0,
            idx=None, counts=True, trace=False, nthreads=None, speeds=None, speed_mask=0):
    """Alg. 1 in FP64.  Returns dict with counts [H,ny,nx] uint32, offgrid [H],
    and with trace=True: trace_k [n,H] uint8, trace_pair [n] int32, trace_cell [n,H]."""
    x0, y0, cell, nx, ny = grid
    beta = np.ascontiguousarray(beta, np.float32)
    goals = np.ascontiguousarray(goals, np.float32).reshape(-1, 2)
    belief = np.ascontiguousarray(belief, np.float64).reshape(-1)
    B, G = beta.size, goals.shape[0]
    assert belief.size == G * B
    idx_arr = None if idx is None else np.ascontiguousarray(idx, np.int64)
    n = N if idx_arr is None else idx_arr.size
    cnt = np.zeros((H, ny, nx), np.uint32) if counts else None
    off = np.zeros(H, np.uint32) if counts else None
    tk = np.zeros((n, H), np.uint8) if trace else None
    tp = np.zeros(n, np.int32) if trace else None
    tc = np.zeros((n, H), np.int32) if trace else None
    v = _speeds(speed, speeds)
    rc = lib().orc_predict(K, v.size, v, speed_mask, dt, B, beta, G, goals.reshape(-1), x0, y0,
                           cell, nx, ny,
                           float(z0[0]), float(z0[1]), belief, N, H, seed, human, cycle,
                           idx_arr, 0 if idx_arr is None else idx_arr.size,
                           None if cnt is None else cnt.reshape(-1), off,
                           None if tk is None else tk.reshape(-1), tp,
                           None if tc is None else tc.reshape(-1),
                           nthreads or default_threads())
    _check(rc, "predict")
    return {"counts": cnt, "offgrid": off, "trace_k": tk, "trace_pair": tp, "trace_cell": tc}


def tie_check(*, K, speed, dt, beta, goals, grid, z0, belief, N, H, seed=0, human=0, cycle=0,
              other_pair, other_k, window=1e-6, pair_window=0.0, idx=None, nthreads=None,
              speeds=None, speed_mask=0):
    """Replay particles and classify another implementation's choices:
    status 0 identical, 1 first difference at a heading-CDF tie within `window`
    (or a pair-CDF tie within `pair_window`), 2 unexplained."""
    x0, y0, cell, nx, ny = grid
    beta = np.ascontiguousarray(beta, np.float32)
    goals = np.ascontiguousarray(goals, np.float32).reshape(-1)
    belief = np.ascontiguousarray(belief, np.float64).reshape(-1)
    idx_arr = None if idx is None else np.ascontiguousarray(idx, np.int64)
    n = N if idx_arr is None else idx_arr.size
    st = np.zeros(n, np.int32)
    first = np.zeros(n, np.int32)
    v = _speeds(speed, speeds)
    rc = lib().orc_tie_check(K, v.size, v, speed_mask, dt, beta.size, beta, goals.size // 2,
                             goals, x0, y0, cell,
                             float(z0[0]), float(z0[1]), belief, N, H, seed, human, cycle,
                             idx_arr, 0 if idx_arr is None else idx_arr.size,
                             np.ascontiguousarray(other_pair, np.int32),
                             np.ascontiguousarray(other_k, np.uint8).reshape(-1), window,
                             pair_window, st, first,
                             nthreads or default_threads())
    _check(rc, "tie_check")
    return st, first


def normalize(counts: np.ndarray, N: int) -> np.ndarray:
    """p = count / N, IEEE FP32 division."""
    return np.asarray(counts).astype(np.float32) / np.float32(N)


# ---------------------------------------------------------------- belief update
def recover_controls(K: int, obs: np.ndarray, speed: float = 1.0, dt: float = 1.0, speeds=None):
    """Recovered controls u* = s*K + k* ([n_obs], -1 for a skipped step) and the
    heading margin.  With one speed u* = k* whatever speed and dt are."""
    obs = np.ascontiguousarray(obs, np.float32).reshape(-1, 2)
    n = obs.shape[0] - 1
    ks = np.empty(max(n, 0), np.int32)
    margin = np.empty(max(n, 0), np.float64)
    v = _speeds(speed, speeds)
    _check(lib().orc_recover_controls(K, v.size, v, dt, obs.reshape(-1), n, ks, margin),
           "recover_controls")
    return ks, margin


def uniform_log_belief(G: int, B: int) -> np.ndarray:
    """b^1 = 1 / (|B| |G|) (Sec. III-B), in log space, layout [G][B]."""
    return np.full((G, B), -np.log(G * B), np.float64)


def belief_update(*, K, speed, dt, beta, goals, obs, log_belief=None, sequential=False,
                  speeds=None):
    """Returns (log_belief [G,B], belief [G,B], ell [n_obs,G,B])."""
    beta = np.ascontiguousarray(beta, np.float32)
    goals = np.ascontiguousarray(goals, np.float32).reshape(-1, 2)
    obs = np.ascontiguousarray(obs, np.float32).reshape(-1, 2)
    B, G = beta.size, goals.shape[0]
    lb = uniform_log_belief(G, B) if log_belief is None else np.array(log_belief, np.float64)
    lb = np.ascontiguousarray(lb.reshape(G, B))
    b = np.empty((G, B), np.float64)
    n = obs.shape[0] - 1
    ell = np.empty((max(n, 0), G, B), np.float64)
    v = _speeds(speed, speeds)
    rc = lib().orc_belief_update(K, v.size, v, dt, B, beta, G, goals.reshape(-1), obs.reshape(-1), n,
                                 lb.reshape(-1), b.reshape(-1), ell.reshape(-1), int(sequential))
    _check(rc, "belief_update")
    return lb, b, ell


# --------------------------------------------------------------- log-likelihood
def loglik(*, K, speed, dt, tracks, lengths, goals, log_beta, per_track_beta=False, nthreads=None):
    tracks = np.ascontiguousarray(tracks, np.float32)
    N, T1 = tracks.shape[0], tracks.shape[1]
    lengths = np.ascontiguousarray(lengths, np.int32)
    goals = np.ascontiguousarray(goals, np.float64).reshape(-1, 2)
    log_beta = np.ascontiguousarray(log_beta, np.float64)
    B = log_beta.shape[-1]
    G = goals.shape[0]
    LL = np.empty((N, B, G), np.float64)
    rc = lib().orc_loglik(K, speed, dt, tracks.reshape(-1), lengths, N, T1 - 1, goals.reshape(-1),
                          G, log_beta.reshape(-1), B, int(per_track_beta), LL.reshape(-1),
                          nthreads or default_threads())
    _check(rc, "loglik")
    return LL


def loglik_grad(*, K, speed, dt, tracks, lengths, goals, log_beta, dLL, per_track_beta=False):
    tracks = np.ascontiguousarray(tracks, np.float32)
    N, T1 = tracks.shape[0], tracks.shape[1]
    lengths = np.ascontiguousarray(lengths, np.int32)
    goals = np.ascontiguousarray(goals, np.float64).reshape(-1, 2)
    log_beta = np.ascontiguousarray(log_beta, np.float64)
    B = log_beta.shape[-1]
    G = goals.shape[0]
    dLL = np.ascontiguousarray(dLL, np.float64).reshape(N, B, G)
    dg = np.empty((G, 2), np.float64)
    db = np.empty(log_beta.shape, np.float64)
    rc = lib().orc_loglik_grad(K, speed, dt, tracks.reshape(-1), lengths, N, T1 - 1,
                               goals.reshape(-1), G, log_beta.reshape(-1), B, int(per_track_beta),
                               dLL.reshape(-1), dg.reshape(-1), db.reshape(-1))
    _check(rc, "loglik_grad")
    return dg, db


# ----------------------------------------------------------------- synthetic humans
def simulate_tracks(*, K, speed, dt, frame, start, beta, goal, T, seed=0, stream=0, speeds=None):
    """Returns (lattice [n,T+1,2] int64, positions [n,T+1,2] float32).
    frame = (x0, y0, cell) fixes the lattice."""
    x0, y0, cell = frame
    start = np.ascontiguousarray(start, np.float64).reshape(-1, 2)
    n = start.shape[0]
    beta = np.ascontiguousarray(beta, np.float32).reshape(n)
    goal = np.ascontiguousarray(goal, np.float32).reshape(n, 2)
    lat = np.empty((n, T + 1, 2), np.int64)
    pos = np.empty((n, T + 1, 2), np.float32)
    v = _speeds(speed, speeds)
    rc = lib().orc_simulate_tracks(K, v.size, v, dt, x0, y0, cell, n, T, start.reshape(-1), beta,
                                   goal.reshape(-1), seed, stream, lat.reshape(-1),
                                   pos.reshape(-1))
    _check(rc, "simulate_tracks")
    return lat, pos


# ------------------------------------------------------------ smoothing and union
def smooth(counts: np.ndarray, N: int, sigma: float, radius: int, cells=None,
           nthreads=None) -> np.ndarray:
    """Gaussian-smoothed occupancy (Sec. III-B) as the direct 2-D sum in FP64.
    counts [H, ny, nx] uint32; returns float64 [H, ny, nx], or [len(cells)]
    for flattened (t, y, x) indices `cells`."""
    counts = np.ascontiguousarray(counts, np.uint32)
    H, ny, nx = counts.shape
    idx = None if cells is None else np.ascontiguousarray(cells, np.int64).reshape(-1)
    out = np.empty(counts.size if idx is None else idx.size, np.float64)
    _check(lib().orc_smooth(counts.reshape(-1), H, ny, nx, N, float(sigma), int(radius), idx,
                            0 if idx is None else idx.size, out, nthreads or default_threads()),
           "smooth")
    return out.reshape(counts.shape) if idx is None else out


def union_max(grids) -> np.ndarray:
    """Point-wise maximum over humans of equally shaped float32 grids (Sec. IV-B)."""
    arrs = [np.ascontiguousarray(g, np.float32) for g in grids]
    shape = arrs[0].shape
    assert all(a.shape == shape for a in arrs)
    ptrs = (C.POINTER(C.c_float) * len(arrs))(
        *[a.ctypes.data_as(C.POINTER(C.c_float)) for a in arrs])
    out = np.empty(shape, np.float32)
    _check(lib().orc_union_max(ptrs, len(arrs), arrs[0].size, out.reshape(-1)), "union_max")
    return out


# ------------------------------------------------------------------------ MPPI
PAPER_MPPI_COST = dict(Q=(3.0, 3.0, 10.0, 0.0), Qf=(0.6, 0.6, 2.0, 0.0), R=(2.0, 1.0),
                       w_coll=1000.0, p_coll=0.1)


def mppi(*, z0, goal, U, delta, dt, tau, Q, Qf, R, w_coll=1000.0, p_coll=0.1, c_time=0.0,
         occ=None, grid=None):
    """One MPPI step (Sec. III-C) in FP64.  U [T,2] (a, omega); delta [T,N,2].
    Returns (S [N], U_new [T,2], near [N]: steps within 1e-9 m of a cell edge)."""
    U = np.ascontiguousarray(U, np.float64).reshape(-1, 2)
    T = U.shape[0]
    delta = np.ascontiguousarray(delta, np.float64)
    assert delta.shape[0] == T and delta.shape[2] == 2
    N = delta.shape[1]
    if occ is not None:
        occ = np.ascontiguousarray(occ, np.float32)
        H = occ.shape[0]
        x0, y0, cell, nx, ny = grid
    else:
        H, x0, y0, cell, nx, ny = 0, 0.0, 0.0, 1.0, 1, 1
    S = np.empty(N, np.float64)
    Un = np.empty((T, 2), np.float64)
    near = np.empty(N, np.int32)
    f = lambda v, n: np.ascontiguousarray(v, np.float64).reshape(n)
    _check(lib().orc_mppi(f(z0, 4), f(goal, 4), T, dt, N, U.reshape(-1), delta.reshape(-1),
                          None if occ is None else occ.reshape(-1), H, float(x0), float(y0),
                          float(cell), int(nx), int(ny), f(Q, 4), f(Qf, 4), f(R, 2),
                          float(w_coll), float(p_coll), float(c_time), float(tau), S,
                          Un.reshape(-1), near), "mppi")
    return S, Un, near
