"""PyTorch binding of libcapred.so (the C ABI in include/capred.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory and the current stream.  The
module raises ImportError when the library has not been built -- there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcapred.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2603_01122_amd.build.build() "
                      "(hipcc for gfx950). There is no CPU fallback.")

_lib = C.CDLL(LIB_PATH)

CAP_OK, CAP_E_INVALID, CAP_E_HIP, CAP_E_WORKSPACE, CAP_E_UNSUPPORTED, CAP_E_CAPACITY = \
    0, -1, -2, -3, -4, -5
MAX_K, MAX_B, MAX_G, MAX_J, MAX_SLOTS = 32, 16, 64, 512, 256


class CapError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = _lib.cap_last_error().decode()
        super().__init__(f"{what} failed with status {status}: {msg}")
        self.status = status


CAP_MAX_S = 8


class cap_model(C.Structure):
    _fields_ = [("K", C.c_int32), ("speed", C.c_double), ("dt", C.c_double), ("B", C.c_int32),
                ("beta", C.POINTER(C.c_float)), ("G", C.c_int32),
                ("goals", C.POINTER(C.c_float)), ("n_speeds", C.c_int32),
                ("speeds", C.POINTER(C.c_double)), ("speed_mask", C.c_uint32)]


class cap_mppi_cost(C.Structure):
    _fields_ = [("Q", C.c_double * 4), ("Qf", C.c_double * 4), ("R", C.c_double * 2),
                ("w_coll", C.c_double), ("p_coll", C.c_double), ("c_time", C.c_double),
                ("tau", C.c_double)]


class cap_grid(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("cell", C.c_double), ("nx", C.c_int32),
                ("ny", C.c_int32)]


class cap_plan_config(C.Structure):
    _fields_ = [("n_slots", C.c_int32), ("K", C.c_int32), ("speed", C.c_double),
                ("dt", C.c_double), ("max_obs", C.c_int32), ("ring", C.c_int32),
                ("block_threads", C.c_int32), ("particles_per_thread", C.c_int32),
                ("lds_bytes", C.c_int32), ("grid_blocks", C.c_int32),
                ("max_smooth_radius", C.c_int32), ("n_speeds", C.c_int32),
                ("speeds", C.c_double * CAP_MAX_S)]


class cap_slot_desc(C.Structure):
    _fields_ = [("human_id", C.c_uint32), ("N", C.c_int32), ("H", C.c_int32), ("B", C.c_int32),
                ("beta", C.POINTER(C.c_float)), ("G", C.c_int32),
                ("goals", C.POINTER(C.c_float)), ("grid", cap_grid),
                ("last_xy", C.c_float * 2), ("counts_dev", C.c_void_p),
                ("offgrid_dev", C.c_void_p), ("probs_dev", C.c_void_p),
                ("log_belief_dev", C.c_void_p), ("belief_dev", C.c_void_p),
                ("reset_belief", C.c_int32), ("smooth_radius", C.c_int32),
                ("smooth_sigma", C.c_double), ("speed_mask", C.c_uint32)]


_vp, _i32, _u32, _u64, _i64, _d, _sz = (C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64,
                                        C.c_int64, C.c_double, C.c_size_t)


def _sig(name, restype, *argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(argtypes)
    return f


_sig("cap_abi_version", _i32)
_sig("cap_last_error", C.c_char_p)
_sig("cap_device_cu_count", _i32)
_sig("cap_belief_update", _i32, C.POINTER(cap_model), _vp, _i32, _vp, _vp, _vp)
_sig("cap_belief_reset", _i32, _i32, _i32, _vp, _vp)
_sig("cap_predict_occupancy", _i32, C.POINTER(cap_model), C.POINTER(cap_grid),
     C.POINTER(C.c_double), _vp, _i32, _i32, _u64, _u32, _u32, _vp, _vp, _vp, _vp, _vp)
_sig("cap_normalize", _i32, _vp, _i64, _i32, _vp, _vp)
_sig("cap_smooth_occupancy", _i32, _vp, _i32, _i32, _i32, _i32, C.c_double, _i32, _vp, _vp)
_sig("cap_union_max", _i32, C.POINTER(_vp), _i32, _i64, _vp, _vp)
_sig("cap_mppi_step", _i32, C.POINTER(C.c_double), C.POINTER(C.c_double), _i32, _d, _i32, _vp, _vp,
     _vp, _i32, _vp, C.POINTER(cap_mppi_cost), _vp, _vp)
_sig("cap_simulate_tracks", _i32, _i32, _d, _i32, C.POINTER(C.c_double), _d, _d, _d, _d, _i32,
     _i32, _vp, _vp, _vp, _u64, _u32, _vp, _vp, _vp)
_sig("cap_loglik", _i32, _i32, _d, _d, _vp, _vp, _i32, _i32, _vp, _i32, _vp, _i32, _i32, _vp, _vp)
_sig("cap_loglik_backward", _i32, _i32, _d, _d, _vp, _vp, _i32, _i32, _vp, _i32, _vp, _i32, _i32,
     _vp, _vp, _vp, _vp, _sz, _vp)
_sig("cap_loglik_backward_workspace", _sz, _i32, _i32, _i32, _i32)
_sig("cap_loglik_backward_noalloc", _i32, _i32, _d, _d, _vp, _vp, _i32, _i32, _vp, _i32, _vp, _i32,
     _i32, _vp, _vp, _vp, _vp)
_sig("cap_philox_blocks", _i32, _i64, _u32, _u32, _u32, _u32, _u64, _vp, _vp)
_sig("cap_probe", _i32, _i32, _i64, _i32, _vp, _vp)
_sig("cap_probe_global_atomic", _i32, _i64, _i32, _vp, _i32, _vp)
_sig("cap_copy", _i32, _vp, _vp, _sz, _vp)
EXPORTED = ["cap_probe", "cap_probe_global_atomic", "cap_copy", "cap_philox_blocks", "cap_abi_version", "cap_last_error", "cap_device_cu_count", "cap_belief_update",
            "cap_belief_reset", "cap_predict_occupancy", "cap_normalize", "cap_simulate_tracks",
            "cap_loglik", "cap_loglik_backward", "cap_loglik_backward_workspace",
            "cap_loglik_backward_noalloc",
            "cap_smooth_occupancy", "cap_union_max", "cap_mppi_step"]
if hasattr(_lib, "cap_plan_create"):
    _sig("cap_plan_create", _i32, C.POINTER(cap_plan_config), C.POINTER(_vp))
    _sig("cap_plan_destroy", None, _vp)
    _sig("cap_plan_set_slot", _i32, _vp, _i32, C.POINTER(cap_slot_desc))
    _sig("cap_plan_clear_slot", _i32, _vp, _i32)
    _sig("cap_plan_set_speed_mask", _i32, _vp, _i32, _u32)
    _sig("cap_plan_reset_belief", _i32, _vp, _i32)
    _sig("cap_plan_stage_obs", _i32, _vp, _i32, _vp, _i32)
    _sig("cap_plan_stage_obs_many", _i32, _vp, _i32, _vp, _vp)
    _sig("cap_plan_run", _i32, _vp, _u64, _u32, _vp)
    _sig("cap_plan_run_plain", _i32, _vp, _u64, _u32, _vp)
    _sig("cap_plan_set_union", _i32, _vp, C.POINTER(cap_grid), _i32, _vp)
    _sig("cap_plan_sync", _i32, _vp)
    _sig("cap_plan_stats", _i32, _vp, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i32))
    _sig("cap_plan_tuning", _i32, _vp, C.POINTER(cap_plan_config))
    _sig("cap_plan_replay_rollout", _i32, _vp, _vp, _vp, _vp)
    _sig("cap_plan_tile_split", _i32, C.POINTER(_i32), _i32, _i32, _i32, _i32, C.POINTER(_i32))
    EXPORTED += ["cap_plan_replay_rollout", "cap_plan_create", "cap_plan_destroy", "cap_plan_set_slot",
                 "cap_plan_clear_slot", "cap_plan_stage_obs", "cap_plan_stage_obs_many",
                 "cap_plan_run",
                 "cap_plan_run_plain", "cap_plan_sync", "cap_plan_stats", "cap_plan_tuning",
                 "cap_plan_set_speed_mask", "cap_plan_reset_belief", "cap_plan_tile_split",
                 "cap_plan_set_union"]


def _check(rc: int, what: str):
    if rc != CAP_OK:
        raise CapError(rc, what)


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _ptr(t: Optional[torch.Tensor], dtype: torch.dtype, name: str, shape=None) -> Optional[int]:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


@dataclasses.dataclass
class Model:
    """Human model of Sec. III-A: K headings at speed v (or at each of `speeds`,
    controls u = s K + k), step dt, beta grid, goals; speed_mask (bit s, 0 = all)
    restricts the prediction to some speeds."""
    K: int
    speed: float
    dt: float
    beta: np.ndarray     # float32 [B]
    goals: np.ndarray    # float32 [G, 2] metres
    speeds: Optional[np.ndarray] = None   # float64 [S] m/s, or None for the one speed
    speed_mask: int = 0

    def __post_init__(self):
        self.beta = np.ascontiguousarray(self.beta, np.float32).reshape(-1)
        self.goals = np.ascontiguousarray(self.goals, np.float32).reshape(-1, 2)
        if self.speeds is not None:
            self.speeds = np.ascontiguousarray(self.speeds, np.float64).reshape(-1)

    @property
    def B(self):
        return int(self.beta.size)

    @property
    def G(self):
        return int(self.goals.shape[0])

    @property
    def S(self):
        return 1 if self.speeds is None else int(self.speeds.size)

    @property
    def U(self):
        return self.K * self.S

    def c(self) -> cap_model:
        m = cap_model(self.K, float(self.speed), float(self.dt), self.B,
                      self.beta.ctypes.data_as(C.POINTER(C.c_float)), self.G,
                      self.goals.ctypes.data_as(C.POINTER(C.c_float)))
        if self.speeds is not None:
            m.n_speeds = self.speeds.size
            m.speeds = self.speeds.ctypes.data_as(C.POINTER(C.c_double))
        m.speed_mask = int(self.speed_mask)
        return m


def model_of(h) -> Model:
    """Model of a scenes.Human."""
    return Model(h.K, h.speed, h.dt, h.beta, h.goals)


def grid_c(grid: Sequence) -> cap_grid:
    x0, y0, cell, nx, ny = grid
    return cap_grid(float(x0), float(y0), float(cell), int(nx), int(ny))


def abi_version() -> int:
    return _lib.cap_abi_version()


def device_cu_count() -> int:
    return _lib.cap_device_cu_count()


# ----------------------------------------------------------------- belief
def belief_reset(log_belief: torch.Tensor, stream=None):
    G, B = log_belief.shape
    _check(_lib.cap_belief_reset(G, B, _ptr(log_belief, torch.float64, "log_belief"),
                                 _stream(stream)), "cap_belief_reset")
    return log_belief


def belief_update(model: Model, obs: torch.Tensor, log_belief: torch.Tensor,
                  belief: Optional[torch.Tensor] = None, stream=None):
    """Eq. (beta_update) over the transitions of obs [n+1, 2]; log_belief [G, B]
    is updated in place; belief (optional) receives exp(log posterior)."""
    m = model.c()
    n_obs = obs.shape[0] - 1
    _ptr(log_belief, torch.float64, "log_belief", (model.G, model.B))
    _check(_lib.cap_belief_update(C.byref(m), _ptr(obs, torch.float32, "obs", (n_obs + 1, 2)),
                                  n_obs, log_belief.data_ptr(),
                                  _ptr(belief, torch.float64, "belief", (model.G, model.B)),
                                  _stream(stream)), "cap_belief_update")
    return log_belief, belief


# ----------------------------------------------------------------- prediction
def predict_occupancy(model: Model, grid: Sequence, z0: Sequence[float], belief: torch.Tensor,
                      N: int, H: int, seed: int = 0, human_id: int = 0, cycle: int = 0,
                      counts: Optional[torch.Tensor] = None,
                      offgrid: Optional[torch.Tensor] = None, trace: bool = False, stream=None):
    """Alg. 1 for one human.  Returns dict(counts [H,ny,nx] int32-view of uint32,
    offgrid [H], trace_k [N,H] uint8, trace_pair [N] int32)."""
    g = grid_c(grid)
    dev = belief.device
    if counts is None:
        counts = torch.empty((H, g.ny, g.nx), dtype=torch.int32, device=dev)
    if offgrid is None:
        offgrid = torch.empty(H, dtype=torch.int32, device=dev)
    tk = torch.empty((N, H), dtype=torch.uint8, device=dev) if trace else None
    tp = torch.empty(N, dtype=torch.int32, device=dev) if trace else None
    m = model.c()
    z = (C.c_double * 2)(float(z0[0]), float(z0[1]))
    _check(_lib.cap_predict_occupancy(
        C.byref(m), C.byref(g), z, _ptr(belief, torch.float64, "belief", (model.G, model.B)),
        N, H, seed, human_id, cycle, _ptr(counts, torch.int32, "counts", (H, g.ny, g.nx)),
        _ptr(offgrid, torch.int32, "offgrid", (H,)), _ptr(tk, torch.uint8, "trace_k"),
        _ptr(tp, torch.int32, "trace_pair"), _stream(stream)), "cap_predict_occupancy")
    return {"counts": counts, "offgrid": offgrid, "trace_k": tk, "trace_pair": tp}


def normalize(counts: torch.Tensor, N: int, probs: Optional[torch.Tensor] = None, stream=None):
    """p = count / N (FP32)."""
    if probs is None:
        probs = torch.empty(counts.shape, dtype=torch.float32, device=counts.device)
    _check(_lib.cap_normalize(_ptr(counts, torch.int32, "counts"), counts.numel(), N,
                              _ptr(probs, torch.float32, "probs", tuple(counts.shape)),
                              _stream(stream)), "cap_normalize")
    return probs


def smooth_occupancy(counts: torch.Tensor, N: int, sigma: float = 1.0, radius: int = 3,
                     probs: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Gaussian-smoothed probabilities of a [H, ny, nx] count stack (FP32)."""
    if counts.dim() != 3:
        raise ValueError("counts must be [H, ny, nx]")
    H, ny, nx = counts.shape
    if probs is None:
        probs = torch.empty(counts.shape, dtype=torch.float32, device=counts.device)
    _check(_lib.cap_smooth_occupancy(_ptr(counts, torch.int32, "counts"), H, ny, nx, N,
                                     float(sigma), int(radius),
                                     _ptr(probs, torch.float32, "probs", tuple(counts.shape)),
                                     _stream(stream)), "cap_smooth_occupancy")
    return probs


def union_max(grids: Sequence[torch.Tensor], out: Optional[torch.Tensor] = None,
              stream=None) -> torch.Tensor:
    """Point-wise maximum over equally shaped FP32 grids on one device."""
    if not grids:
        raise ValueError("at least one grid is needed")
    shape = tuple(grids[0].shape)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=grids[0].device)
    ptrs = (_vp * len(grids))(*[_ptr(g, torch.float32, "grid", shape) for g in grids])
    _check(_lib.cap_union_max(ptrs, len(grids), grids[0].numel(),
                              _ptr(out, torch.float32, "out", shape), _stream(stream)),
           "cap_union_max")
    return out


PAPER_MPPI_COST = dict(Q=(3.0, 3.0, 10.0, 0.0), Qf=(0.6, 0.6, 2.0, 0.0), R=(2.0, 1.0),
                       w_coll=1000.0, p_coll=0.1)


def mppi_step(z0: Sequence[float], goal: Sequence[float], U: torch.Tensor, delta: torch.Tensor,
              dt: float, tau: float, Q=(3.0, 3.0, 10.0, 0.0), Qf=(0.6, 0.6, 2.0, 0.0),
              R=(2.0, 1.0), w_coll: float = 1000.0, p_coll: float = 0.1, c_time: float = 0.0,
              occ: Optional[torch.Tensor] = None, grid: Optional[Sequence] = None,
              S: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """One MPPI step (Sec. III-C) of the 4-D Dubins robot against the predicted
    grids occ [H, ny, nx] (FP32, or None): updates U [T, 2] (FP64, in place)
    from perturbations delta [T, N, 2] (FP64) and returns the costs S [N]."""
    if U.dim() != 2 or U.shape[1] != 2 or delta.dim() != 3 or delta.shape[0] != U.shape[0] \
            or delta.shape[2] != 2:
        raise ValueError("U must be [T, 2] and delta [T, N, 2]")
    T, N = U.shape[0], delta.shape[1]
    if S is None:
        S = torch.empty(N, dtype=torch.float64, device=U.device)
    cost = cap_mppi_cost((C.c_double * 4)(*Q), (C.c_double * 4)(*Qf), (C.c_double * 2)(*R),
                         float(w_coll), float(p_coll), float(c_time), float(tau))
    H = 0 if occ is None else occ.shape[0]
    g = None if occ is None else C.byref(grid_c(grid))
    if occ is not None and tuple(occ.shape[1:]) != (int(grid[4]), int(grid[3])):
        raise ValueError("occ must be [H, ny, nx] of the grid")
    _check(_lib.cap_mppi_step((C.c_double * 4)(*[float(x) for x in z0]),
                              (C.c_double * 4)(*[float(x) for x in goal]), T, float(dt), N,
                              _ptr(U, torch.float64, "U"), _ptr(delta, torch.float64, "delta"),
                              _ptr(occ, torch.float32, "occ"), H, g, C.byref(cost),
                              _ptr(S, torch.float64, "S", (N,)), _stream(stream)),
           "cap_mppi_step")
    return S


def philox_blocks(n: int, c0: int, c1: int, c2: int, c3: int, seed: int, device="cuda",
                  stream=None) -> torch.Tensor:
    """Raw Philox4x32-10 blocks for counters (c0+i, c1, c2, c3): int32 view [n, 4]."""
    out = torch.empty((n, 4), dtype=torch.int32, device=device)
    _check(_lib.cap_philox_blocks(n, c0, c1, c2, c3, seed, out.data_ptr(), _stream(stream)),
           "cap_philox_blocks")
    return out


PROBE_KINDS = {"fma": 0, "exp2": 1, "sqrt": 2, "rcp": 3, "mul64": 4, "lds_atomic": 5, "mix": 6}


def probe(kind: str, iters: int, blocks: int, sink: torch.Tensor, stream=None):
    """Launches one throughput probe (8 chains x iters ops per thread, 256 threads/block)."""
    _check(_lib.cap_probe(PROBE_KINDS[kind], iters, blocks, _ptr(sink, torch.float32, "sink"),
                          _stream(stream)), "cap_probe")


def probe_global_atomic(iters: int, blocks: int, counts: torch.Tensor, stream=None):
    """Launches the device-scope atomic-add probe (8 chains x iters adds per
    thread, 256 threads/block) over counts, an int32 buffer of 2^k words."""
    n = counts.numel()
    if n & (n - 1) or not 64 <= n <= 1 << 30:
        raise ValueError("counts must hold 2^k words, k in [6, 30]")
    _check(_lib.cap_probe_global_atomic(iters, blocks, _ptr(counts, torch.int32, "counts"),
                                        n.bit_length() - 1, _stream(stream)),
           "cap_probe_global_atomic")


def copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    _check(_lib.cap_copy(src.data_ptr(), dst.data_ptr(), src.numel() * src.element_size(),
                         _stream(stream)), "cap_copy")


def simulate_tracks(K: int, speed: float, dt: float, frame: Sequence[float],
                    start: torch.Tensor, beta: torch.Tensor, goal: torch.Tensor, T: int,
                    seed: int = 0, stream_id: int = 0, stream=None, speeds=None):
    """Synthetic humans.  start [n,2] f64, beta [n] f32, goal [n,2] f32 (device);
    speeds (host, m/s) selects the multi-speed control set.
    Returns (lattice [n,T+1,2] int32, positions [n,T+1,2] f32)."""
    n = start.shape[0]
    lat = torch.empty((n, T + 1, 2), dtype=torch.int32, device=start.device)
    pos = torch.empty((n, T + 1, 2), dtype=torch.float32, device=start.device)
    x0, y0, cell = frame
    v = None if speeds is None else np.ascontiguousarray(speeds, np.float64).reshape(-1)
    _check(_lib.cap_simulate_tracks(K, speed, 0 if v is None else v.size,
                                    None if v is None else v.ctypes.data_as(C.POINTER(C.c_double)),
                                    dt, x0, y0, cell, n, T,
                                    _ptr(start, torch.float64, "start", (n, 2)),
                                    _ptr(beta, torch.float32, "beta", (n,)),
                                    _ptr(goal, torch.float32, "goal", (n, 2)), seed, stream_id,
                                    lat.data_ptr(), pos.data_ptr(), _stream(stream)),
           "cap_simulate_tracks")
    return lat, pos


# ----------------------------------------------------------------- log-likelihood
def _ll_args(K, speed, dt, tracks, lengths, goals, log_beta):
    N, T1, _ = tracks.shape
    G = goals.shape[0]
    per_track = 1 if log_beta.dim() == 2 else 0
    B = log_beta.shape[-1]
    if per_track and log_beta.shape[0] != N:
        raise ValueError("per-track log_beta must be [N, B]")
    return (K, float(speed), float(dt), _ptr(tracks, torch.float32, "tracks"),
            _ptr(lengths, torch.int32, "lengths", (N,)), N, T1 - 1,
            _ptr(goals, torch.float32, "goals", (G, 2)), G,
            _ptr(log_beta, torch.float32, "log_beta"), B, per_track)


def loglik(K, speed, dt, tracks, lengths, goals, log_beta, stream=None) -> torch.Tensor:
    """LL [N, B, G] FP64 (product form of Eq. beta_update over each track)."""
    args = _ll_args(K, speed, dt, tracks, lengths, goals, log_beta)
    N, G, B = args[5], args[8], args[10]
    LL = torch.empty((N, B, G), dtype=torch.float64, device=tracks.device)
    _check(_lib.cap_loglik(*args, LL.data_ptr(), _stream(stream)), "cap_loglik")
    return LL


def loglik_backward(K, speed, dt, tracks, lengths, goals, log_beta, dLL, stream=None):
    """(dgoals [G,2] FP64, dlog_beta like log_beta in FP64)."""
    args = _ll_args(K, speed, dt, tracks, lengths, goals, log_beta)
    N, G, B, per_track = args[5], args[8], args[10], args[11]
    dLL = dLL.to(torch.float64).contiguous()
    _ptr(dLL, torch.float64, "dLL", (N, B, G))
    dg = torch.empty((G, 2), dtype=torch.float64, device=tracks.device)
    db = torch.empty(tuple(log_beta.shape), dtype=torch.float64, device=tracks.device)
    ws_bytes = _lib.cap_loglik_backward_workspace(N, G, B, per_track)
    ws = torch.empty(max(ws_bytes, 8), dtype=torch.uint8, device=tracks.device)
    _check(_lib.cap_loglik_backward(*args, dLL.data_ptr(), dg.data_ptr(), db.data_ptr(),
                                    ws.data_ptr(), ws_bytes, _stream(stream)),
           "cap_loglik_backward")
    return dg, db


def loglik_backward_noalloc(K, speed, dt, tracks, lengths, goals, log_beta, dLL, dgoals,
                            dlog_beta, stream=None):
    """loglik_backward into caller-provided outputs (dgoals [G,2], dlog_beta
    shaped like log_beta, both FP64) through the library's allocation-free
    entry point: nothing is allocated on the device by this call."""
    args = _ll_args(K, speed, dt, tracks, lengths, goals, log_beta)
    N, G, B = args[5], args[8], args[10]
    _ptr(dLL, torch.float64, "dLL", (N, B, G))
    _ptr(dgoals, torch.float64, "dgoals", (G, 2))
    _ptr(dlog_beta, torch.float64, "dlog_beta", tuple(log_beta.shape))
    _check(_lib.cap_loglik_backward_noalloc(*args, dLL.data_ptr(), dgoals.data_ptr(),
                                            dlog_beta.data_ptr(), _stream(stream)),
           "cap_loglik_backward_noalloc")


class LogLik(torch.autograd.Function):
    """LL = LogLik.apply(goals [G,2] f32, log_beta [B] or [N,B] f32, tracks, lengths, K, speed, dt);
    backward through the hand-written adjoint kernel."""

    @staticmethod
    def forward(ctx, goals, log_beta, tracks, lengths, K, speed, dt):
        goals_c = goals.detach().contiguous()
        lb_c = log_beta.detach().contiguous()
        ctx.save_for_backward(goals_c, lb_c, tracks, lengths)
        ctx.model = (K, speed, dt)
        return loglik(K, speed, dt, tracks, lengths, goals_c, lb_c)

    @staticmethod
    def backward(ctx, dLL):
        goals, lb, tracks, lengths = ctx.saved_tensors
        K, speed, dt = ctx.model
        dg, db = loglik_backward(K, speed, dt, tracks, lengths, goals, lb, dLL)
        return dg.to(goals.dtype), db.to(lb.dtype), None, None, None, None, None


# ----------------------------------------------------------------- batched plans
@dataclasses.dataclass
class SlotBuffers:
    """Device buffers of one admitted human (ring of per-cycle outputs)."""
    counts: torch.Tensor      # [ring, H, ny, nx] int32 (uint32 counts)
    probs: Optional[torch.Tensor]   # [ring, H, ny, nx] f32
    offgrid: torch.Tensor     # [ring, H] int32
    log_belief: torch.Tensor  # [G, B] f64 state
    belief: torch.Tensor      # [ring, G, B] f64 posterior

    @staticmethod
    def allocate(model: Model, grid, H: int, ring: int, probs: bool = True, device="cuda"):
        nx, ny = int(grid[3]), int(grid[4])
        return SlotBuffers(
            torch.empty((ring, H, ny, nx), dtype=torch.int32, device=device),
            torch.empty((ring, H, ny, nx), dtype=torch.float32, device=device) if probs else None,
            torch.empty((ring, H), dtype=torch.int32, device=device),
            torch.empty((model.G, model.B), dtype=torch.float64, device=device),
            torch.empty((ring, model.G, model.B), dtype=torch.float64, device=device))


def tile_split(units, particles_per_thread: int, resident_blocks: int, cus: int) -> np.ndarray:
    """Tiles of the persistent launch per human: counts [n, 3] of tiles holding
    P, P/2 and P/4 units of block_threads particles (host computation)."""
    u = np.ascontiguousarray(units, np.int32).reshape(-1)
    out = np.zeros((u.size, 3), np.int32)
    _check(_lib.cap_plan_tile_split(u.ctypes.data_as(C.POINTER(C.c_int32)), u.size,
                                    particles_per_thread, resident_blocks, cus,
                                    out.ctypes.data_as(C.POINTER(C.c_int32))),
           "cap_plan_tile_split")
    return out


class Plan:
    """Batched many-human prediction (cap_plan_*): one persistent rollout launch
    per cycle, captured in hipGraphs, with continuous admission of humans."""

    def __init__(self, K: int, speed: float, dt: float, n_slots: int, max_obs: int = 1,
                 ring: int = 2, block_threads: int = 0, particles_per_thread: int = 0,
                 lds_bytes: int = 0, grid_blocks: int = 0, max_smooth_radius: int = 0,
                 speeds=None):
        cfg = cap_plan_config(n_slots, K, speed, dt, max_obs, ring, block_threads,
                              particles_per_thread, lds_bytes, grid_blocks, max_smooth_radius)
        if speeds is not None:
            v = np.ascontiguousarray(speeds, np.float64).reshape(-1)
            if v.size > CAP_MAX_S:
                raise ValueError(f"at most {CAP_MAX_S} speeds")
            cfg.n_speeds = v.size
            for i, x in enumerate(v):
                cfg.speeds[i] = float(x)
        h = C.c_void_p()
        _check(_lib.cap_plan_create(C.byref(cfg), C.byref(h)), "cap_plan_create")
        self._h = h
        self.K, self.speed, self.dt, self.ring = K, speed, dt, ring
        self.speeds = None if speeds is None else np.asarray(speeds, np.float64).reshape(-1)
        self.n_slots = n_slots
        self.buffers = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.cap_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tuning(self) -> dict:
        c = cap_plan_config()
        _check(_lib.cap_plan_tuning(self._h, C.byref(c)), "cap_plan_tuning")
        out = {f: getattr(c, f) for f, _ in cap_plan_config._fields_}
        out["speeds"] = list(out["speeds"])[:c.n_speeds]
        return out

    def admit(self, slot: int, human_id: int, model: Model, grid, N: int, H: int,
              last_xy, buffers: SlotBuffers, reset_belief: bool = True,
              smooth: Optional[Tuple[float, int]] = None):
        """smooth = (sigma, radius) in cells asks for Gaussian-smoothed probabilities."""
        if model.K != self.K:
            raise ValueError("model K differs from the plan's")
        if (model.speeds is None) != (self.speeds is None) or (
                model.speeds is not None and not np.array_equal(model.speeds, self.speeds)):
            raise ValueError("model speeds differ from the plan's control set")
        desc = cap_slot_desc()
        desc.human_id = human_id
        desc.N, desc.H, desc.B, desc.G = N, H, model.B, model.G
        desc.beta = model.beta.ctypes.data_as(C.POINTER(C.c_float))
        desc.goals = model.goals.ctypes.data_as(C.POINTER(C.c_float))
        desc.grid = grid_c(grid)
        desc.last_xy[0], desc.last_xy[1] = float(last_xy[0]), float(last_xy[1])
        desc.counts_dev = _ptr(buffers.counts, torch.int32, "counts",
                               (self.ring, H, int(grid[4]), int(grid[3])))
        desc.offgrid_dev = _ptr(buffers.offgrid, torch.int32, "offgrid", (self.ring, H))
        desc.probs_dev = _ptr(buffers.probs, torch.float32, "probs")
        desc.log_belief_dev = _ptr(buffers.log_belief, torch.float64, "log_belief",
                                   (model.G, model.B))
        desc.belief_dev = _ptr(buffers.belief, torch.float64, "belief",
                               (self.ring, model.G, model.B))
        desc.reset_belief = 1 if reset_belief else 0
        if smooth is not None:
            desc.smooth_sigma, desc.smooth_radius = float(smooth[0]), int(smooth[1])
        desc.speed_mask = int(model.speed_mask)
        _check(_lib.cap_plan_set_slot(self._h, slot, C.byref(desc)), "cap_plan_set_slot")
        self.buffers[slot] = buffers

    def retire(self, slot: int):
        _check(_lib.cap_plan_clear_slot(self._h, slot), "cap_plan_clear_slot")
        self.buffers.pop(slot, None)

    def set_speed_mask(self, slot: int, mask: int):
        _check(_lib.cap_plan_set_speed_mask(self._h, slot, int(mask)), "cap_plan_set_speed_mask")

    def reset_belief(self, slot: int):
        _check(_lib.cap_plan_reset_belief(self._h, slot), "cap_plan_reset_belief")

    def set_union(self, frame, H: int, union: Optional[torch.Tensor]):
        """From the next cycle on, write the point-wise maximum of the
        probabilities of the slots whose grid is `frame` into union[cycle % ring]
        ([ring, H, ny, nx] FP32); union=None switches the stage off."""
        if union is None:
            _check(_lib.cap_plan_set_union(self._h, None, 0, None), "cap_plan_set_union")
            self._union = None
            return
        g = grid_c(frame)
        ptr = _ptr(union, torch.float32, "union", (self.ring, H, int(frame[4]), int(frame[3])))
        _check(_lib.cap_plan_set_union(self._h, C.byref(g), H, ptr), "cap_plan_set_union")
        self._union = union

    def stage(self, slot: int, xy):
        # called for every human every cycle: the array's address is passed as a
        # plain integer (a ctypes POINTER object costs several microseconds)
        a = np.ascontiguousarray(xy, np.float32).reshape(-1, 2)
        _check(_lib.cap_plan_stage_obs(self._h, slot, a.ctypes.data, a.shape[0]),
               "cap_plan_stage_obs")

    def stage_many(self, slots, xy):
        """One new position per listed slot in one call: slots [n] int32,
        xy [n, 2] (metres)."""
        sl = np.ascontiguousarray(slots, np.int32).reshape(-1)
        a = np.ascontiguousarray(xy, np.float32).reshape(-1, 2)
        if a.shape[0] != sl.size:
            raise ValueError("one position per slot")
        _check(_lib.cap_plan_stage_obs_many(self._h, sl.size, sl.ctypes.data, a.ctypes.data),
               "cap_plan_stage_obs_many")

    def run(self, seed: int, cycle: int, stream=None):
        _check(_lib.cap_plan_run(self._h, seed, cycle, _stream(stream)), "cap_plan_run")

    def run_plain(self, seed: int, cycle: int, stream=None):
        _check(_lib.cap_plan_run_plain(self._h, seed, cycle, _stream(stream)),
               "cap_plan_run_plain")

    def replay_rollout(self, stream=None, ev_start=None, ev_end=None):
        _check(_lib.cap_plan_replay_rollout(
            self._h, _stream(stream), None if ev_start is None else ev_start.cuda_event,
            None if ev_end is None else ev_end.cuda_event), "cap_plan_replay_rollout")

    def sync(self):
        _check(_lib.cap_plan_sync(self._h), "cap_plan_sync")

    def stats(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int32()
        _check(_lib.cap_plan_stats(self._h, C.byref(a), C.byref(b), C.byref(c)), "cap_plan_stats")
        return a.value, b.value, c.value
