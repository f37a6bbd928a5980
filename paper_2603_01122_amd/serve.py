"""Fixed-rate serving loop with continuous batching over a batched plan.

The paper predicts its k humans one after another every cycle (Sec. IV-B);
here every cycle is one batched plan run (hipGraphs: belief update of every
active human from its newest observation, grid clear, one persistent rollout
launch, normalisation).  Humans arrive and leave while cycles are in flight:

* admission -- an arriving human waits until a slot is free and the particle
  budget (total particles in flight per cycle, which bounds the cycle time)
  has room for its N; it then joins at the next cycle boundary;
* departure -- a departing human leaves the next cycle at once, but its slot
  is only reused once every cycle in flight that included it has completed:
  a newcomer's buffer views are shaped by its own G, B, H and grid, so its
  ring entries and belief rows can overlap the departed human's, which those
  cycles are still reading and writing;
* overlap -- consecutive cycles go to alternating streams and use alternating
  ring entries of every per-cycle buffer, so cycle c+1 can start on the device
  while cycle c is still running; only the tiny belief updates are ordered;
* latency -- a cycle's latency is the time from its release tick until the
  host observes its completion event (polled, never a blocking wait);
* host pauses -- Python's full garbage collections walk every tracked object
  of the process (tens of milliseconds once torch is loaded) and land on
  whichever cycle triggers them; the server freezes the heap that exists when
  it starts (gc.freeze) so that later collections only walk what the loop
  itself creates, and it keeps a bounded history of cycle records.

Results are keyed by (human id, cycle, seed) alone, so a human's grids are the
same whether it is served alone or in any mix.  Slot buffers are allocated
once up front (no allocation in the loop).
"""
from __future__ import annotations

import collections
import dataclasses
import gc
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import capred


@dataclasses.dataclass
class HumanRequest:
    hid: int
    model: capred.Model
    grid: Sequence
    N: int
    H: int
    last_xy: Sequence[float]
    log_belief: Optional[np.ndarray] = None   # carried state; None = uniform prior
    smooth: Optional[Tuple[float, int]] = None  # (sigma, radius) cells: smoothed probabilities


@dataclasses.dataclass
class CycleRecord:
    cycle: int
    release: float
    done_event: torch.cuda.Event
    humans: List[int]
    particle_steps: int
    completed: Optional[float] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.completed is None else self.completed - self.release


class Admission:
    """Host-side admission control of the serving loop (no device work, so it
    is testable on its own).  A human waits in FIFO order until a slot is free
    and the particle budget has room for its N; a request that does not fit
    does not block later ones that do.  A departed human's slot is reused only
    once every completion predicate handed to depart() reports done (the
    cycles in flight that still read or write the slot's buffers)."""

    def __init__(self, n_slots: int, budget: Optional[int] = None):
        self.free: List[int] = list(range(n_slots))
        self.retiring: List[Tuple[int, List]] = []
        self.waiting: collections.deque = collections.deque()
        self.budget = budget
        self.in_use = 0
        self.active: Dict[int, Tuple[int, int]] = {}   # hid -> (slot, N)

    def submit(self, r) -> None:
        self.waiting.append(r)

    def depart(self, hid: int, busy: Sequence = ()) -> Optional[int]:
        """Removes `hid` (active or waiting).  busy: completion predicates
        (objects with .query()) of the in-flight work that uses its slot.
        Returns the slot it held, or None if it was still waiting."""
        if hid in self.active:
            s, n = self.active.pop(hid)
            self.in_use -= n
            busy = list(busy)
            if busy:
                self.retiring.append((s, busy))
            else:
                self.free.append(s)
            return s
        self.waiting = collections.deque(r for r in self.waiting if r.hid != hid)
        return None

    def reclaim(self) -> None:
        keep = []
        for s, evs in self.retiring:
            if all(e.query() for e in evs):
                self.free.append(s)
            else:
                keep.append((s, evs))
        self.retiring = keep

    def admit(self) -> List[Tuple[int, object]]:
        """Reclaims finished slots, then admits waiting requests in order while
        slots and budget allow; returns [(slot, request)]."""
        self.reclaim()
        out, kept = [], collections.deque()
        while self.waiting:
            r = self.waiting.popleft()
            fits = self.budget is None or self.in_use + r.N <= self.budget
            if self.free and fits:
                s = self.free.pop(0)
                self.active[r.hid] = (s, r.N)
                self.in_use += r.N
                out.append((s, r))
            else:
                kept.append(r)
        self.waiting = kept
        return out


def latency_summary(latencies: Sequence[float], period: float) -> dict:
    """p50 / p99 / max latency (ms) and deadline misses (latency > period) of
    completed cycles (seconds)."""
    lat = np.asarray(latencies, np.float64)
    return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
            "max_ms": round(float(lat.max()) * 1e3, 4), "cycles": int(lat.size),
            "deadline_ms": round(period * 1e3, 3),
            "deadline_misses": int(np.count_nonzero(lat > period))}


class Server:
    def __init__(self, K: int, speed: float, dt: float, n_slots: int, max_H: int, max_nx: int,
                 max_ny: int, max_G: int, max_B: int, ring: int = 2, n_streams: int = 2,
                 particle_budget: Optional[int] = None, seed: int = 0, probs: bool = True,
                 tuning: Optional[dict] = None, max_smooth_radius: int = 0, speeds=None,
                 stationary: Optional[Tuple[float, int]] = None,
                 goal_departure: Optional[float] = None, device="cuda",
                 freeze_gc: bool = True, history: int = 1 << 16,
                 union: Optional[Tuple[Sequence, int]] = None, clock=time.perf_counter,
                 first_cycle: int = 0):
        """stationary = (eps, mask): a human whose newest observed step is shorter
        than eps metres is predicted with the allowed speeds `mask` only (Q = -inf
        for the others, Sec. IV-B) until it moves again.  goal_departure = r: a
        human that was within r metres of one of its goals and is now farther
        from all of them gets a uniform belief before the next update (Sec. IV-B).
        The paper specifies neither detector; these are the simplest readings.
        Both are fixed at construction (with neither, a cycle skips the
        per-human detection bookkeeping).
        freeze_gc: gc.freeze() once the server is built (see the module notes).
        history: how many of the latest CycleRecords `records` keeps.
        union = (frame, H): every cycle also writes, inside its graph, the
        point-wise maximum of the probabilities of the humans whose grid is
        `frame` (the planner's single occupancy map of Sec. IV-B), read with
        union_grid(cycle).  clock: the host clock of release and completion
        times (seconds).  first_cycle: number of the first cycle (a server that
        resumes humans from carried state continues the cycle numbering, which
        keys the random streams)."""
        tuning = tuning or {}
        self.plan = capred.Plan(K, speed, dt, n_slots, max_obs=1, ring=ring,
                                max_smooth_radius=max_smooth_radius, speeds=speeds, **tuning)
        self.stationary = stationary
        self.goal_departure = goal_departure
        self._last_xy: Dict[int, np.ndarray] = {}
        self._at_goal: Dict[int, bool] = {}
        self._masked: Dict[int, bool] = {}
        self.K, self.ring, self.seed = K, ring, seed
        self.max = (max_H, max_nx, max_ny, max_G, max_B)
        cells = max_H * max_nx * max_ny
        self.pool_counts = torch.zeros((n_slots, ring * cells), dtype=torch.int32, device=device)
        self.pool_probs = (torch.zeros((n_slots, ring * cells), dtype=torch.float32, device=device)
                           if probs else None)
        self.pool_off = torch.zeros((n_slots, ring * max_H), dtype=torch.int32, device=device)
        self.pool_lb = torch.zeros((n_slots, max_G * max_B), dtype=torch.float64, device=device)
        self.pool_b = torch.zeros((n_slots, ring * max_G * max_B), dtype=torch.float64,
                                  device=device)
        self.pool_union = None
        if union is not None:
            frame, uH = union
            self.pool_union = torch.zeros((ring, uH, int(frame[4]), int(frame[3])),
                                          dtype=torch.float32, device=device)
            self.plan.set_union(frame, uH, self.pool_union)
        self.adm = Admission(n_slots, particle_budget)
        self.clock = clock
        self.slot_of: Dict[int, int] = {}
        self.req: Dict[int, HumanRequest] = {}
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        # The pools are filled on the caller's current stream; the serving streams
        # must not start before those fills (nor before any later host-driven
        # write to a slot's buffers, see _after_current_stream).
        self._dep: Optional[torch.cuda.Event] = None
        self._after_current_stream()
        self.cycle = int(first_cycle)
        self.records: collections.deque = collections.deque(maxlen=max(1, history))
        self._pending: collections.deque = collections.deque()
        if freeze_gc:
            gc.collect()
            gc.freeze()

    # ----------------------------------------------------------- admission
    def submit(self, r: HumanRequest):
        H, nx, ny = r.H, int(r.grid[3]), int(r.grid[4])
        if H > self.max[0] or nx > self.max[1] or ny > self.max[2] or r.model.G > self.max[3] \
                or r.model.B > self.max[4] or r.model.K != self.K:
            raise ValueError(f"human {r.hid} exceeds the slot capacity of this server")
        self.adm.submit(r)

    @property
    def waiting(self) -> collections.deque:
        return self.adm.waiting

    def depart(self, hid: int):
        for d in (self._last_xy, self._at_goal, self._masked):
            d.pop(hid, None)
        busy = [r.done_event for r in self._pending if hid in r.humans]
        s = self.adm.depart(hid, busy)
        if s is not None:
            self.slot_of.pop(hid)
            self.req.pop(hid)
            self.plan.retire(s)

    def _views(self, s: int, r: HumanRequest) -> capred.SlotBuffers:
        R, H, nx, ny = self.ring, r.H, int(r.grid[3]), int(r.grid[4])
        G, B = r.model.G, r.model.B
        n = R * H * ny * nx
        return capred.SlotBuffers(
            self.pool_counts[s, :n].view(R, H, ny, nx),
            None if self.pool_probs is None else self.pool_probs[s, :n].view(R, H, ny, nx),
            self.pool_off[s, :R * H].view(R, H),
            self.pool_lb[s, :G * B].view(G, B),
            self.pool_b[s, :R * G * B].view(R, G, B))

    def _admit_waiting(self):
        for s, r in self.adm.admit():
            buf = self._views(s, r)
            if r.log_belief is not None:
                buf.log_belief.copy_(torch.as_tensor(r.log_belief, dtype=torch.float64))
                self._after_current_stream()
            self.plan.admit(s, r.hid, r.model, r.grid, r.N, r.H, r.last_xy, buf,
                            reset_belief=r.log_belief is None, smooth=r.smooth)
            self.slot_of[r.hid] = s
            self.req[r.hid] = r

    # ----------------------------------------------------------- cycles
    def step(self, observations: Dict[int, Sequence[float]], release: Optional[float] = None,
             plain: bool = False) -> CycleRecord:
        """Admits waiting humans, stages each active human's new position and
        launches one cycle (batched, or the per-human reference if plain)."""
        self._admit_waiting()
        seen = [(hid, xy) for hid, xy in observations.items() if hid in self.slot_of]
        if seen:
            # one library call for all humans, validated as a whole: a rejected
            # observation leaves every human's state as it was
            self.plan.stage_many([self.slot_of[hid] for hid, _ in seen], [xy for _, xy in seen])
        if self.stationary is not None or self.goal_departure is not None:
            for hid, xy in seen:
                self._detect(hid, xy)
        stream = self.streams[self.cycle % len(self.streams)]
        if self._dep is not None:
            for st in self.streams:
                st.wait_event(self._dep)
            self._dep = None
        ev = torch.cuda.Event()
        # the library takes the stream itself: no switch of torch's current stream
        if plain:
            self.plan.run_plain(self.seed, self.cycle, stream)
        else:
            self.plan.run(self.seed, self.cycle, stream)
        ev.record(stream)
        rec = CycleRecord(self.cycle, self.clock() if release is None else release, ev,
                          sorted(self.slot_of), sum(self.req[h].N * self.req[h].H
                                                    for h in self.slot_of))
        self.records.append(rec)
        self._pending.append(rec)
        self.cycle += 1
        return rec

    def _after_current_stream(self):
        """Orders the next cycle after the work queued so far on the current stream."""
        self._dep = torch.cuda.Event()
        self._dep.record(torch.cuda.current_stream())

    def _detect(self, hid: int, xy):
        """Stationary and goal-departure detection on the newest observation."""
        s = self.slot_of[hid]
        z = np.asarray(xy, np.float64)
        prev = self._last_xy.get(hid)
        if prev is None:
            prev = np.asarray(self.req[hid].last_xy, np.float64)
        if self.stationary is not None:
            eps, slow = self.stationary
            still = bool(np.hypot(*(z - prev)) < eps)
            if still != self._masked.get(hid, False):
                self.plan.set_speed_mask(s, slow if still else self.req[hid].model.speed_mask)
                self._masked[hid] = still
        if self.goal_departure is not None:
            d = np.min(np.hypot(*(self.req[hid].model.goals.astype(np.float64) - z).T))
            near = bool(d <= self.goal_departure)
            if self._at_goal.get(hid, False) and not near:
                self.plan.reset_belief(s)
            self._at_goal[hid] = near
        self._last_xy[hid] = z

    def poll(self) -> int:
        """Marks finished cycles (non-blocking); returns how many are still pending."""
        now = self.clock()
        while self._pending and self._pending[0].done_event.query():
            self._pending.popleft().completed = now
        return len(self._pending)

    def drain(self):
        while self.poll():
            time.sleep(20e-6)

    def grids(self, hid: int, cycle: int):
        """(counts [H,ny,nx], probs, offgrid, posterior [G,B]) of `hid` at `cycle`
        (valid until that ring entry is reused)."""
        s = self.slot_of[hid]
        r = self.req[hid]
        b = self._views(s, r)
        e = cycle % self.ring
        return (b.counts[e], None if b.probs is None else b.probs[e], b.offgrid[e], b.belief[e])

    def union_grid(self, cycle: int) -> torch.Tensor:
        """[H, ny, nx] union of `cycle` (valid until its ring entry is reused)."""
        return self.pool_union[cycle % self.ring]

    def log_belief(self, hid: int) -> torch.Tensor:
        """`hid`'s log posterior [G, B] after the newest cycle that has run
        (read it once that cycle is complete, e.g. after drain())."""
        s = self.slot_of[hid]
        return self._views(s, self.req[hid]).log_belief

    def close(self):
        self.plan.sync()
        self.plan.close()


def run_paced(server, obs_fn, n_cycles: int, rate_hz: float = 125.0, progress=None,
              before_step=None, clock=time.perf_counter, sleep=time.sleep) -> np.ndarray:
    """Fixed-rate loop: cycle c is released at t0 + c/rate; between ticks the
    host polls the completion events back to back while a cycle is in flight
    (a completion is seen within one poll, a few microseconds; a sleep of
    tens of microseconds would overshoot by the kernel's timer slack) and
    sleeps otherwise, waking 150 us before the tick and spinning to it.  A
    cycle that outlasts the period does not hold back the next tick's launch.
    before_step(c) (optional) runs after the release tick, before
    the cycle is launched (arrivals and departures: their host work counts in
    that cycle's latency).  obs_fn(c) -> {hid: xy}.  Returns latencies (s);
    the server must stamp completions with the same clock."""
    period = 1.0 / rate_hz
    t0 = clock() + 2 * period
    recs = []
    for c in range(n_cycles):
        tick = t0 + c * period
        while True:
            pending = server.poll()
            now = clock()
            if now >= tick:
                break
            if not pending and tick - now > 200e-6:
                sleep(min(tick - now - 150e-6, 1e-3))
        if before_step is not None:
            before_step(c)
        recs.append(server.step(obs_fn(c), release=tick))
        if progress and (c + 1) % progress[0] == 0:
            progress[1](c + 1)
    server.drain()
    return np.array([r.latency for r in recs], np.float64)
