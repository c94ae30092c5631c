"""Continuous batching of many reduced simulations on one GPU.

Requests (a simulation plus a number of latent steps) arrive over time. The server admits
them in arrival order while a slot and the HBM budget allow (each sim's device memory is
nsf_sim_bytes of its descriptor), keeps every admitted sim's latent, weights and grid
resident, and advances all of them together: one tick is one nsf_step_batch call, i.e.
one replay of a graph whose kernels run over the union of the sims' work. Sims that
finish retire at a tick boundary and free their memory, so requests that arrived
meanwhile join the next tick. Each tick's device time is recorded with HIP events (the
step latency every sim in that tick sees); results are read when a sim retires.

The compute backend is injected so the scheduling logic can be exercised without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Deque, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    workload: object              # anything Sim() accepts (synth.Workload)
    steps: int
    keep_positions: bool = False  # read the decoded positions at retirement


@dataclasses.dataclass
class Result:
    rid: int
    arrival_s: float
    admitted_s: float
    finished_s: float
    steps: int
    n_particles: int
    z: np.ndarray
    flags: int
    positions: Optional[np.ndarray] = None


class GpuBackend:
    """The real device path: Sim objects from the HIP library, batched steps."""

    def __init__(self, precision: str = "bf16", decode_every_step: bool = True):
        import torch

        from . import _abi
        from .sim import Sim, step_batch
        self.torch = torch
        self.Sim, self._step_batch, self._abi = Sim, step_batch, _abi
        self.precision = precision
        self.decode = decode_every_step
        self.stream = torch.cuda.Stream()
        self._events: List = []

    def sim_bytes(self, w) -> int:
        # size the arena without creating: the descriptor is built inside Sim, so use a
        # throwaway probe of the same arithmetic (nsf_sim_bytes) through Sim's builder
        return self.Sim.bytes_for(w, self.precision)

    def create(self, w):
        return self.Sim(w, precision=self.precision, decode_every_step=self.decode, stream=self.stream)

    def step(self, sims) -> None:
        t = self.torch
        a, b = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        a.record(self.stream)
        self._step_batch(sims, 1, stream=self.stream)
        b.record(self.stream)
        self._events.append((a, b))

    def tick_ms(self) -> List[float]:
        self.stream.synchronize()
        return [a.elapsed_time(b) for a, b in self._events]

    def wait_behind(self, depth: int) -> None:
        """Keep the host at most `depth` ticks ahead of the device."""
        if len(self._events) > depth:
            self._events[-1 - depth][1].synchronize()

    def finish(self, sim, keep_positions: bool):
        z, _, st = sim.latent(stream=self.stream)
        status, flags = sim.flags(stream=self.stream)
        pos = None
        if keep_positions:
            pos = sim.buffer(self._abi.NSF_BUF_XDEC).reshape(3, -1).cpu().numpy().copy()
        sim.close()
        return z, flags, pos


class Server:
    def __init__(self, backend, hbm_budget_bytes: int, max_slots: int = 1024,
                 max_ahead: int = 2, clock: Callable[[], float] = time.perf_counter):
        self.backend = backend
        self.budget = int(hbm_budget_bytes)
        self.max_slots = int(max_slots)
        self.max_ahead = max_ahead
        self.clock = clock
        self.pending: Deque[Request] = collections.deque()
        self.waiting: Deque[Request] = collections.deque()
        self.active: Dict[int, dict] = {}
        self.results: List[Result] = []
        self.ticks: List[dict] = []   # per tick: active rids and count
        self.used = 0
        self.peak_used = 0
        self.peak_active = 0

    def submit(self, reqs: List[Request]) -> None:
        for r in sorted(reqs, key=lambda q: q.arrival_s):
            self.pending.append(r)

    # ---- one scheduling round --------------------------------------------------------
    def _admit(self, now: float) -> None:
        while self.pending and self.pending[0].arrival_s <= now:
            self.waiting.append(self.pending.popleft())
        while self.waiting and len(self.active) < self.max_slots:
            req = self.waiting[0]
            need = self.backend.sim_bytes(req.workload)
            if need > self.budget:
                raise ValueError(f"request {req.rid} needs {need} bytes, more than the budget")
            if self.used + need > self.budget:
                break   # FIFO: wait for memory to free up
            self.waiting.popleft()
            sim = self.backend.create(req.workload)
            self.active[req.rid] = dict(req=req, sim=sim, bytes=need, done=0, admitted=now)
            self.used += need
        self.peak_used = max(self.peak_used, self.used)
        self.peak_active = max(self.peak_active, len(self.active))

    def _retire(self, now: float) -> None:
        for rid in [k for k, a in self.active.items() if a["done"] >= a["req"].steps]:
            a = self.active.pop(rid)
            z, flags, pos = self.backend.finish(a["sim"], a["req"].keep_positions)
            self.used -= a["bytes"]
            req = a["req"]
            self.results.append(Result(rid, req.arrival_s, a["admitted"], now, a["done"],
                                       int(req.workload.X.shape[1]), z, flags, pos))

    def run(self, t0: Optional[float] = None) -> dict:
        """Serve every submitted request; returns the run's statistics."""
        start = self.clock() if t0 is None else t0
        while self.pending or self.waiting or self.active:
            now = self.clock() - start
            self._retire(now)
            self._admit(now)
            if not self.active:
                if self.pending:   # idle until the next arrival
                    nxt = self.pending[0].arrival_s
                    while self.clock() - start < nxt:
                        pass
                continue
            sims = [a["sim"] for a in self.active.values()]
            self.backend.step(sims)
            self.ticks.append(dict(n=len(sims), t=now))
            for a in self.active.values():
                a["done"] += 1
            self.backend.wait_behind(self.max_ahead)
        wall = self.clock() - start
        return self.stats(wall)

    def stats(self, wall: float) -> dict:
        tick_ms = np.asarray(self.backend.tick_ms(), np.float64)
        n = np.asarray([t["n"] for t in self.ticks], np.int64)
        # every (sim, step) pair sees its tick's device time as its step latency
        lat = np.repeat(tick_ms, n) if len(tick_ms) else np.zeros(1)
        steps = int(sum(r.steps for r in self.results))
        pts = int(sum(r.steps * r.n_particles for r in self.results))
        wait = np.asarray([r.admitted_s - r.arrival_s for r in self.results] or [0.0])
        return dict(requests=len(self.results), wall_s=wall, ticks=len(tick_ms),
                    latent_steps=steps, latent_steps_per_s=steps / wall,
                    decoded_pts_per_s=pts / wall,
                    p50_step_ms=float(np.percentile(lat, 50)),
                    p99_step_ms=float(np.percentile(lat, 99)),
                    p50_admission_wait_s=float(np.percentile(wait, 50)),
                    p99_admission_wait_s=float(np.percentile(wait, 99)),
                    peak_active=self.peak_active, peak_bytes=self.peak_used,
                    budget_bytes=self.budget,
                    failed=int(sum(1 for r in self.results if r.flags)))
