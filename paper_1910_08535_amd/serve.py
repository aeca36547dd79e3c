"""Continuous-batching server for right-hand-side and explicit-step requests.

The request loop itself is native (iga_server_* in the library, see include/iga.h):
admission by device memory; iterations in which every admitted request with axes of at
least 3p+1 elements advances together (a right-hand side once, an explicit step by one
step per iteration); a context cache bound to a pool of streams for the other requests;
event-based completion.  This module replays
arrivals in wall-clock time, hands each arriving group of requests to the library in one
call, and records latencies:

* Requests arrive over time (``inputs.request_stream``: Poisson arrivals, 1D/2D/3D,
  p in {2,3}, RHS = fused Petrov-Galerkin apply (mass and Laplacian rows), STEP =
  nsteps explicit steps of u_t = Lap u + sin source with dt = h_min^2 / 64).
* A request may bring its coefficients already on the device (Request.u; the server
  then updates them in place for a step request) and its two output arrays
  (Request.out, shape (2,) + coefficient shape); otherwise they are drawn from its seed
  and allocated at submission.
* Latency of a request = time its completion is observed - its arrival time.

Results do not depend on the mix: a request gives the bits it gives alone on a context
(the same row arithmetic and the same band rows; tests check equality bit for bit).
"""
from __future__ import annotations

import collections
import gc
import time
from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np

from . import iga
from .inputs import Request


@dataclass
class Record:
    req: Request
    t_arrive: float = -1.0          # arrival, in the library's clock (seconds)
    t_done: float = -1.0            # completion observed, same clock
    gauss_points: int = 0
    hbm_bytes: int = 0
    tensors: Tuple = ()             # (u, mass rows, Laplacian rows) or (u,)
    batch_launch: int = -1          # index of the batch launch that ran it, -1 for none

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


def request_shape(req: Request) -> Tuple[int, ...]:
    return tuple(n + req.p for n in reversed(req.ne))


def context_bytes(dim: int, p: int, ne: Tuple[int, ...]) -> int:
    """Approximate device bytes of a mesh context (Gauss-point and band tables)."""
    w = 2 * p + 1
    total = 0
    for n in ne[:dim]:
        total += 8 * (n * (p + 2) + (n + p) * (5 * w + 4))
    return total


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


class MeshCache:
    """Contexts by (dim, p, element counts), least recently used first out once their
    device bytes exceed a limit; new contexts are bound round-robin to the given streams."""

    def __init__(self, streams, limit_bytes: int = 16 << 30):
        self.streams = streams
        self.limit = limit_bytes
        self.bytes = 0
        self.next = 0
        self.meshes: "collections.OrderedDict[tuple, iga.Mesh]" = collections.OrderedDict()

    def get(self, dim: int, p: int, ne: Tuple[int, ...]) -> "iga.Mesh":
        key = (dim, p, ne)
        m = self.meshes.get(key)
        if m is not None:
            self.meshes.move_to_end(key)
            return m
        s = self.streams[self.next % len(self.streams)] if self.streams else None
        self.next += 1
        m = iga.Mesh(dim, p, ne, (p + 1,) * dim, stream=s)
        self.meshes[key] = m
        self.bytes += context_bytes(dim, p, ne)
        while self.bytes > self.limit and len(self.meshes) > 1:
            (d, q, n), old = self.meshes.popitem(last=False)
            self.bytes -= context_bytes(d, q, n)
            old.close()
        return m

    def close(self) -> None:
        for m in self.meshes.values():
            m.close()
        self.meshes.clear()
        self.bytes = 0


def batched(req: Request) -> bool:
    """Whether the library's batched iterations take the request: every axis has at least
    3p+1 elements (the size limits of a mesh context aside)."""
    return all(n >= 3 * req.p + 1 for n in req.ne)


def footprint(req: Request) -> int:
    """Bytes a request holds while in flight, as the library counts them against its
    budget: coefficients plus both outputs (RHS), or coefficients plus the step's work
    buffer; for a batched request also its own band tables (M and D rows per axis, and the
    step's scale and source rows; in 1D only the step's source rows)."""
    n = 1
    for d in request_shape(req):
        n *= d
    b = (3 if req.kind == "rhs" else 2) * 8 * n
    if batched(req):
        w = 2 * req.p + 1
        step = req.kind != "rhs"
        if req.dim == 1:
            b += 8 * (req.ne[0] + req.p) if step else 0
        else:
            b += 8 * sum((m + req.p) * (2 * w + (2 if step else 0)) for m in req.ne)
    return b


class Server:
    def __init__(self, budget_bytes: int = 200 * 10**9, streams: int = 4,
                 mesh_cache_bytes: int = 16 << 30, keep_outputs: bool = False):
        import torch
        self.torch = torch
        self.native = iga.NativeServer(streams, budget_bytes, mesh_cache_bytes)
        self.keep = keep_outputs
        self.gen = torch.Generator(device="cuda")
        self.done: List[Record] = []
        self.live: Dict[int, Record] = {}

    @property
    def used(self) -> int:
        return self.native.stats()[0]

    @property
    def peak(self) -> int:
        return self.native.stats()[1]

    def _tensors(self, req: Request):
        torch = self.torch
        shape = request_shape(req)
        u = req.u
        if u is None:
            self.gen.manual_seed(req.seed)
            u = torch.randn(shape, dtype=torch.float64, device="cuda", generator=self.gen)
        if req.kind != "rhs":
            return (u,)
        out = getattr(req, "out", None)
        if out is None:
            out = torch.empty((2,) + shape, dtype=torch.float64, device="cuda")
        return (u, out[0], out[1])

    def prepare(self, reqs: List[Request]):
        """The library's request records of `reqs` and their bookkeeping, built before any
        timing (the client's side of a submission: device buffers and descriptors)."""
        recs = np.zeros(len(reqs), dtype=self.native.dtype)
        records = []
        fresh = False
        for k, req in enumerate(reqs):
            fresh = fresh or req.u is None or (req.kind == "rhs" and getattr(req, "out", None) is None)
            tens = self._tensors(req)
            r = recs[k]
            r["kind"] = iga.REQ_RHS if req.kind == "rhs" else iga.REQ_STEP
            r["dim"], r["p"] = req.dim, req.p
            r["ne"][: req.dim] = req.ne
            r["ne"][req.dim:] = 1
            r["u"] = tens[0].data_ptr()
            if req.kind == "rhs":
                r["mass_out"], r["lap_out"] = tens[1].data_ptr(), tens[2].data_ptr()
            else:
                h = min(1.0 / n for n in req.ne)
                r["nsteps"], r["dt"], r["sin_amp"] = req.nsteps, h * h / 64.0, 1.0
            rec = Record(req=req, tensors=tens)
            rec.gauss_points, rec.hbm_bytes = request_work(req)
            records.append(rec)
        if fresh:   # coefficients drawn or outputs allocated on torch's stream just now
            self.torch.cuda.current_stream().synchronize()
        return recs, records

    def submit(self, reqs: List[Request], arrivals: List[float]) -> None:
        """Hands a group of arrived requests to the library (arrival times in the
        library's clock)."""
        if not reqs:
            return
        recs, records = self.prepare(reqs)
        for rec, t in zip(records, arrivals):
            rec.t_arrive = t
        self._submit(recs, records)

    def _submit(self, recs, records) -> None:
        tickets = self.native.submit(recs)
        for t, rec in zip(tickets.tolist(), records):
            self.live[t] = rec

    def _progress(self) -> int:
        tickets, times, states, launches = self.native.progress()
        for t, tm, st, ln in zip(tickets.tolist(), times.tolist(), states.tolist(), launches.tolist()):
            rec = self.live.pop(t)
            if st != iga.JOB_DONE:
                raise RuntimeError(f"request failed: {rec.req}")
            rec.t_done = tm
            rec.batch_launch = ln
            if not self.keep:
                rec.tensors = ()
            self.done.append(rec)
        return len(tickets)

    # ---- the loop --------------------------------------------------------------------
    def run(self, requests: List[Request], time_scale: float = 1.0) -> Dict[str, float]:
        """Serve `requests` (arrivals replayed in wall-clock time scaled by time_scale,
        every request at once for 0) until all are done; returns latency and throughput
        figures.  The request records are prepared before the clock starts; in the loop a
        group of arrived requests is one library call."""
        order = sorted(requests, key=lambda r: r.t_arrive)
        recs, records = self.prepare(order)
        arrive = [r.t_arrive * time_scale for r in order]
        total = len(order) + len(self.done)
        start = self.native.stats()[3]
        for rec, a in zip(records, arrive):
            rec.t_arrive = start + a
        nxt = 0
        # no collector passes inside the loop: with many live objects one pass takes
        # milliseconds, which would show up as request latency
        collect = gc.isenabled()
        gc.disable()
        try:
            t0 = time.perf_counter()
            while len(self.done) < total:
                now = time.perf_counter() - t0
                end = nxt
                while end < len(order) and arrive[end] <= now:
                    end += 1
                if end > nxt:
                    self._submit(recs[nxt:end], records[nxt:end])
                    nxt = end
                self._progress()
            wall = time.perf_counter() - t0
        finally:
            if collect:
                gc.enable()
        return self.summary(wall)

    def summary(self, wall: float) -> Dict[str, float]:
        lat = sorted(r.latency for r in self.done)
        n = len(lat)
        gp = sum(r.gauss_points for r in self.done)
        by = sum(r.hbm_bytes for r in self.done)

        def pct(q):
            return lat[min(n - 1, int(q * n))] if n else float("nan")

        return {"requests": n, "wall_s": wall, "p50_ms": pct(0.50) * 1e3, "p99_ms": pct(0.99) * 1e3,
                "max_ms": (lat[-1] * 1e3) if n else float("nan"), "GPs": gp / wall,
                "algorithmic_GBs": by / wall / 1e9, "batch_launches": self.native.stats()[2]}

    def close(self) -> None:
        self.torch.cuda.synchronize()
        self.native.close()
