"""Continuous-batching server for right-hand-side and explicit-step requests.

Every computation runs in the library's kernels; this module only schedules them:

* Requests arrive over time (``inputs.request_stream``: Poisson arrivals, 1D/2D/3D,
  p in {2,3}, RHS = fused Petrov-Galerkin apply (mass and Laplacian rows), STEP =
  nsteps explicit steps of u_t = Lap u + sin source with dt = h_min^2 / 64).
* Admission by device memory: a request is admitted, in arrival order, when its
  resident state (coefficients plus outputs or the step's work buffer) fits in the
  budget next to everything admitted and not yet finished; its state stays on the
  device until it completes.
* 2D RHS requests go to the persistent batch kernel (iga_batch).  Whenever no batch
  launch is running and jobs are queued, one launch takes all of them; requests that
  arrive while a launch runs ride the next one (iteration-level continuous batching).
* Explicit steps and 1D/3D RHS requests run on a pool of streams, concurrently with
  the batch launch and with each other; every mesh gets a context (tables built once,
  cached) bound to one stream of the pool.
* Latency of a request = completion time - arrival time (wall clock; completion is
  observed from the HIP events of its launch).

Results do not depend on the mix: a request runs the same kernels with the same
launch geometry alone and among others (tests check equality bit for bit).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

from . import iga
from .inputs import Request


@dataclass
class Record:
    req: Request
    t_admit: float = -1.0
    t_done: float = -1.0
    bytes: int = 0
    gauss_points: int = 0
    hbm_bytes: int = 0
    tensors: Tuple = ()
    ticket: Optional[int] = None    # batch ticket (2D RHS)
    event: object = None            # stream event (others)
    batch_launch: int = -1

    @property
    def latency(self) -> float:
        return self.t_done - self.req.t_arrive


def request_shape(req: Request) -> Tuple[int, ...]:
    return tuple(n + req.p for n in reversed(req.ne))


def request_work(req: Request) -> Tuple[int, int]:
    """(Gauss points, algorithmic HBM bytes) of a request."""
    ncoef = 1
    nel = 1
    for n in req.ne:
        ncoef *= n + req.p
        nel *= n
    gp = nel * (req.p + 1) ** req.dim
    if req.kind == "rhs":
        return gp, 24 * ncoef
    return gp * req.nsteps, 16 * ncoef * req.nsteps


class Server:
    def __init__(self, budget_bytes: int = 200 * 10**9, streams: int = 4, max_batch: int = 4096,
                 batch_rows: int = 8, max_meshes: int = 512, keep_outputs: bool = False):
        import torch
        self.torch = torch
        self.budget = budget_bytes
        self.used = 0
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.batch_stream = torch.cuda.Stream()
        self.batch = iga.Batch(max_jobs=max_batch, stream=self.batch_stream)
        self.batch_rows = batch_rows
        self.meshes: "collections.OrderedDict[tuple, iga.Mesh]" = collections.OrderedDict()
        self.max_meshes = max_meshes
        self.next_stream = 0
        self.keep = keep_outputs
        self.batch_running: List[Record] = []
        self.batch_queued: List[Record] = []
        self.batch_event = None
        self.batch_launches = 0
        # launches on one stream complete in order: one FIFO of records per stream
        self.inflight: Dict[int, "collections.deque[Record]"] = {
            id(st): collections.deque() for st in self.streams}
        self.gen = torch.Generator(device="cuda")
        self.done: List[Record] = []

    # ---- meshes ------------------------------------------------------------------
    def mesh(self, req: Request) -> "iga.Mesh":
        key = (req.dim, req.p, req.ne)
        m = self.meshes.get(key)
        if m is not None:
            self.meshes.move_to_end(key)
            return m
        s = self.streams[self.next_stream % len(self.streams)]
        self.next_stream += 1
        m = iga.Mesh(req.dim, req.p, req.ne, (req.p + 1,) * req.dim, stream=s)
        self.meshes[key] = m
        while len(self.meshes) > self.max_meshes:
            _, old = self.meshes.popitem(last=False)
            old.close()
        return m

    # ---- admission and dispatch -----------------------------------------------------
    def footprint(self, req: Request) -> int:
        n = 1
        for d in request_shape(req):
            n *= d
        return (3 if req.kind == "rhs" else 2) * 8 * n

    def admit(self, req: Request, now: float) -> Optional[Record]:
        need = self.footprint(req)
        if self.used + need > self.budget:
            return None
        torch = self.torch
        rec = Record(req=req, t_admit=now, bytes=need)
        rec.gauss_points, rec.hbm_bytes = request_work(req)
        self.used += need
        shape = request_shape(req)
        gen = self.gen
        gen.manual_seed(req.seed)
        if req.dim == 2 and req.kind == "rhs":
            with torch.cuda.stream(self.batch_stream):
                u = torch.randn(shape, dtype=torch.float64, device="cuda", generator=gen)
                m, l = torch.empty_like(u), torch.empty_like(u)
            rec.tensors = (u, m, l)
            self.batch_queued.append(rec)
            return rec
        mesh = self.mesh(req)
        s = mesh.stream
        with torch.cuda.stream(s):
            u = torch.randn(shape, dtype=torch.float64, device="cuda", generator=gen)
            if req.kind == "rhs":
                m, l = mesh.apply(iga.PG, u)
                rec.tensors = (u, m, l)
            else:
                h = min(1.0 / n for n in req.ne)
                dt = h * h / 64.0
                for _ in range(req.nsteps):
                    mesh.explicit_step(u, dt, sin_amp=1.0, nsteps=1)
                rec.tensors = (u,)
            ev = torch.cuda.Event()
            ev.record(s)
        rec.event = ev
        self.inflight[id(s)].append(rec)
        return rec

    def _flush_batch(self, now: float) -> None:
        if self.batch_running or not self.batch_queued:
            return
        jobs = [(r.req.p, r.req.ne, *r.tensors) for r in self.batch_queued]
        for r in self.batch_queued:
            r.batch_launch = self.batch_launches
        tickets = self.batch.submit(jobs)
        for r, t in zip(self.batch_queued, tickets):
            r.ticket = t
        self.batch.flush()
        ev = self.torch.cuda.Event()
        ev.record(self.batch_stream)
        self.batch_event = ev
        self.batch_running = self.batch_queued
        self.batch_queued = []
        self.batch_launches += 1

    def _complete(self, rec: Record, now: float) -> None:
        rec.t_done = now
        self.used -= rec.bytes
        if not self.keep:
            rec.tensors = ()
        self.done.append(rec)

    def _progress(self, now: float) -> None:
        if self.batch_running and self.batch_event.query():
            for r in self.batch_running:
                self._complete(r, now)
            self.batch_running = []
        for q in self.inflight.values():
            while q and q[0].event.query():
                self._complete(q.popleft(), now)

    # ---- the loop --------------------------------------------------------------------
    def run(self, requests: List[Request], time_scale: float = 1.0) -> Dict[str, float]:
        """Serve `requests` (sorted by arrival; arrivals replayed in wall-clock time scaled
        by time_scale) until all are done; returns latency and throughput figures."""
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrive))
        waiting: "collections.deque[Request]" = collections.deque()
        t0 = time.perf_counter()
        total = len(requests)
        while len(self.done) < total:
            now = time.perf_counter() - t0
            while pending and pending[0].t_arrive * time_scale <= now:
                waiting.append(pending.popleft())
            while waiting:
                if self.admit(waiting[0], now) is None:
                    break
                waiting.popleft()
            self._flush_batch(now)
            self._progress(time.perf_counter() - t0)
        wall = time.perf_counter() - t0
        return self.summary(wall, time_scale)

    def summary(self, wall: float, time_scale: float = 1.0) -> Dict[str, float]:
        lat = sorted((r.t_done - r.req.t_arrive * time_scale) for r in self.done)
        n = len(lat)
        gp = sum(r.gauss_points for r in self.done)
        by = sum(r.hbm_bytes for r in self.done)

        def pct(q):
            return lat[min(n - 1, int(q * n))] if n else float("nan")

        return {"requests": n, "wall_s": wall, "p50_ms": pct(0.50) * 1e3, "p99_ms": pct(0.99) * 1e3,
                "max_ms": (lat[-1] * 1e3) if n else float("nan"), "GPs": gp / wall,
                "algorithmic_GBs": by / wall / 1e9, "batch_launches": self.batch_launches}

    def close(self) -> None:
        self.torch.cuda.synchronize()
        self.batch.close()
        for m in self.meshes.values():
            m.close()
        self.meshes.clear()
