"""Seeded synthetic inputs shared by the GPU tests, the oracle tests and bench.py.

This module holds random numbers and shapes only -- none of the method's
arithmetic -- so that the GPU path and the CPU oracle can be fed identical data
without sharing any code.  Every generator is numpy PCG64 ``default_rng(seed)``.

Array conventions: coefficient arrays are C-ordered (N_z, N_y, N_x) with
N_a = ne_a + p; a Gauss-point table has shape (ne_z*nq_z, ne_y*nq_y, ne_x*nq_x).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np


def coef_shape(ne: Sequence[int], p: int) -> Tuple[int, ...]:
    return tuple(int(n) + p for n in reversed(list(ne)))


def gauss_shape(ne: Sequence[int], nq: Sequence[int]) -> Tuple[int, ...]:
    return tuple(int(n) * int(q) for n, q in zip(reversed(list(ne)), reversed(list(nq))))


def normal_coefs(ne: Sequence[int], p: int, seed: int) -> np.ndarray:
    """N(0,1) B-spline coefficients."""
    return np.random.default_rng(seed).standard_normal(coef_shape(ne, p))


def uniform_table(shape: Sequence[int], seed: int, scale: float = 1.0) -> np.ndarray:
    """scale * U(-1, 1), one value per Gauss point."""
    return scale * np.random.default_rng(seed).uniform(-1.0, 1.0, size=tuple(shape))


# ---- the five workloads ----------------------------------------------------

@dataclass
class Laplace1D:
    """1D Laplace, quadratic C1, 64 elements, 3-point Gauss; f = sin(pi x) + 0.1 U(-1,1)
    per Gauss point (the sine part is evaluated by each side at its own Gauss points;
    the noise comes from here, drawn in Gauss-grid order)."""
    p: int = 2
    ne: int = 64
    nq: int = 3
    seed: int = 1

    def noise(self) -> np.ndarray:
        return uniform_table((self.ne * self.nq,), self.seed, 0.1)


@dataclass
class Apply2D:
    """2D, quadratic C1, 1024 x 1024 elements, 3x3 Gauss; N(0,1) coefficients."""
    p: int = 2
    ne: Tuple[int, int] = (1024, 1024)
    nq: Tuple[int, int] = (3, 3)
    seed: int = 2

    def coefs(self) -> np.ndarray:
        return normal_coefs(self.ne, self.p, self.seed)


@dataclass
class Heat3D:
    """3D heat u_t = Lap u + f, cubic C2, 128^3 elements, 4^3 Gauss, dt = 1e-6,
    100 explicit steps, u0 = N(0,1), f = sin(pi x) sin(pi y) sin(pi z)."""
    p: int = 3
    ne: Tuple[int, int, int] = (128, 128, 128)
    nq: Tuple[int, int, int] = (4, 4, 4)
    dt: float = 1e-6
    nsteps: int = 100
    sin_amp: float = 1.0
    seed: int = 3

    def coefs(self) -> np.ndarray:
        return normal_coefs(self.ne, self.p, self.seed)


@dataclass
class BatchJob:
    p: int
    ne: Tuple[int, int]   # (n, m) = elements along (x, y)


def batch_jobs(count: int = 256, seed: int = 4, lo: int = 32, hi: int = 1024
               ) -> Tuple[List[BatchJob], List[np.ndarray]]:
    """256 independent 2D problems: p in {2,3}, then n, m in U{lo..hi}, then
    N(0,1) coefficients of shape (m+p, n+p), drawn in that order."""
    rng = np.random.default_rng(seed)
    ps = rng.integers(2, 4, size=count)
    ns = rng.integers(lo, hi + 1, size=count)
    ms = rng.integers(lo, hi + 1, size=count)
    jobs, coefs = [], []
    for k in range(count):
        p, n, m = int(ps[k]), int(ns[k]), int(ms[k])
        jobs.append(BatchJob(p=p, ne=(n, m)))
        coefs.append(rng.standard_normal((m + p, n + p)))
    return jobs, coefs


@dataclass
class Request:
    t_arrive: float        # seconds from the start of the stream
    kind: str              # "rhs" or "step"
    dim: int
    p: int
    ne: Tuple[int, ...]    # elements per axis (x, y, z)
    nsteps: int            # explicit steps (0 for rhs)
    seed: int              # seed of this request's coefficients
    u: object = None       # the coefficients already on the device (optional)
    out: object = None     # RHS: its two output arrays on the device, (2,) + u.shape (optional)


def request_stream(rate: float = 2000.0, seconds: float = 10.0, seed: int = 5,
                   max_1d: int = 1_000_000, max_2d: int = 2048, max_3d: int = 192
                   ) -> List[Request]:
    """Poisson arrivals; kind 50/50 rhs / explicit step (nsteps ~ U{1..10});
    dim ~ U{1,2,3}; p ~ U{2,3}; element counts log-uniform per axis
    (1D [1e3, max_1d], 2D [32, max_2d], 3D [16, max_3d])."""
    rng = np.random.default_rng(seed)
    out: List[Request] = []
    t = 0.0
    k = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        kind = "rhs" if rng.random() < 0.5 else "step"
        dim = int(rng.integers(1, 4))
        p = int(rng.integers(2, 4))
        lo, hi = {1: (1e3, max_1d), 2: (32, max_2d), 3: (16, max_3d)}[dim]
        ne = tuple(int(round(np.exp(rng.uniform(np.log(lo), np.log(hi))))) for _ in range(dim))
        nsteps = int(rng.integers(1, 11)) if kind == "step" else 0
        out.append(Request(t, kind, dim, p, ne, nsteps, int(rng.integers(0, 2**31 - 1))))
        k += 1
    return out
