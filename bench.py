"""Benchmark: Gauss-points/s of the Petrov-Galerkin generation on one MI355X.

Workload (default): 2D Laplace, quadratic C1 tensor B-splines, 1024 x 1024 elements on
the unit square, 3 x 3 Gauss points per element, FP64, seeded N(0,1) coefficients.
One step = one fused matrix-free apply with support spans:
    mass_r = int_{S_r} u_h,   lap_r = int_{S_r} Lap u_h     (both written)
which touches every one of the 9,437,184 Gauss points' contributions once
(sum-factorized).  Algorithmic HBM bytes per step: read u (1026^2 doubles) and write
two row arrays = 24 B per coefficient = 25.26 MB.

The K timed steps run as one replay of a HIP graph holding K launches, cycling
through enough distinct (u, mass, lap) buffer sets (>= 512 MB) that the 256 MB
Infinity Cache cannot hold the working set: inputs are resident in HBM when the
timed region starts.

Prints one JSON line (rank 0).  --gpus above 1 exits: the path runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, vendor figure
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector, vendor figure
GP_C2 = 1024 * 1024 * 9
BYTES_C2 = 1026 * 1026 * 24


def kernel_source_hash(kernel: str = "apply2d") -> str:
    from paper_1910_08535_amd.profiling import kernel_source_hash as h
    return h(kernel)


def copy_probe(mib: int) -> None:
    """A plain device copy of known size (for scaling the HBM byte counters of a
    profiling run of this script)."""
    import torch
    n = mib * 2**20 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def measured_traffic(workload: str, kernel: str = None):
    """HBM bytes per launch from a committed rocprofv3 counter summary of the workload
    (profiles/traffic_<workload>*.json: one per tile that was profiled) taken on the
    current kernel sources and on the named kernel; else None."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"traffic_{workload}*.json"))):
        with open(path) as fh:
            rec = json.load(fh)
        if rec.get("kernel_source_hash") != kernel_source_hash(rec.get("family", "apply2d")):
            continue
        if kernel is not None and kernel not in rec.get("kernel", ""):
            continue
        return rec.get("bytes_per_launch")
    return None


def cpu_baseline(args) -> dict:
    """The oracle (test infrastructure) on the host cores: the full 1024^2 workload,
    mass rows and Laplacian rows (two oracle passes over every Gauss point), best of 3."""
    from oracle import oracle as orc
    from paper_1910_08535_amd import inputs
    c = inputs.Apply2D()
    u = c.coefs()
    pb = orc.Problem(dim=2, p=c.p, ne=c.ne, nq=c.nq)
    best = None
    for _ in range(3):
        t0 = time.perf_counter()
        orc.rhs(pb, orc.PG, u, alpha=1.0)
        orc.rhs(pb, orc.PG, u, beta=1.0)
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    out = {"value": GP_C2 / best, "unit": "GP/s", "cores": orc.num_threads(), "kind": "oracle",
           "sample": "full 1024x1024 p=2 workload (mass and Laplacian PG rows), best of 3 runs, "
                     f"{best:.3f} s each"}
    if not args.no_cpu_others:
        out["other_workloads"] = cpu_others()
    return out


def cpu_others() -> dict:
    """The oracle on bounded samples of the other workloads, in Gauss points per second
    (each about a few seconds on the host cores): the 1D Laplace rows (all forms), one
    explicit step of the 3D heat problem at 64^3 (the 128^3 step takes 20-50 s), and the
    first 8 problems of the batched draw."""
    import numpy as np

    from oracle import oracle as orc
    from paper_1910_08535_amd import inputs
    res = {}
    c1 = inputs.Laplace1D()
    pb = orc.Problem(dim=1, p=c1.p, ne=(c1.ne,), nq=(c1.nq,))
    u = np.random.default_rng(c1.seed).standard_normal(pb.coef_shape())
    reps = 200
    t0 = time.perf_counter()
    for _ in range(reps):
        for form in (orc.GALERKIN_BYPARTS, orc.GALERKIN_LAPLACIAN, orc.PG):
            orc.rhs(pb, form, u, alpha=1.0)
    dt = time.perf_counter() - t0
    res["c1_laplace_1d"] = {"GPs": 3 * reps * c1.ne * c1.nq / dt,
                            "sample": f"64 elements, p=2: RHS rows of the three forms x {reps}"}
    c3 = inputs.Heat3D()
    ne = (64, 64, 64)
    pb = orc.Problem(dim=3, p=c3.p, ne=ne, nq=c3.nq)
    u = inputs.normal_coefs(ne, c3.p, c3.seed)
    t0 = time.perf_counter()
    orc.explicit_step(pb, u, c3.dt, sin_amp=c3.sin_amp, nsteps=1)
    dt = time.perf_counter() - t0
    res["c3_heat_3d"] = {"GPs": 64 ** 3 * 4 ** 3 / dt,
                         "sample": f"one explicit step at 64^3, p=3, 4^3 Gauss: {dt:.2f} s"}
    jobs, coefs = inputs.batch_jobs()
    gp, t0 = 0, time.perf_counter()
    for job, cf in zip(jobs[:8], coefs[:8]):
        pb = orc.Problem(dim=2, p=job.p, ne=job.ne, nq=(job.p + 1, job.p + 1))
        orc.rhs(pb, orc.PG, cf, alpha=1.0)
        orc.rhs(pb, orc.PG, cf, beta=1.0)
        gp += job.ne[0] * job.ne[1] * (job.p + 1) ** 2
    dt = time.perf_counter() - t0
    res["c4_batched"] = {"GPs": gp / dt,
                         "sample": f"first 8 of the 256 problems, mass and Laplacian rows each: {dt:.2f} s"}
    return res


def large_2d(args, stream) -> dict:
    """The same fused apply at 4096^2 elements, p = 2 (403 MB per buffer set, two sets
    alternating), on the autotuned tile: a launch long enough that ramp-up and tail no
    longer dominate.  HIP events around a graph of 40 launches."""
    import torch
    from paper_1910_08535_amd import iga

    n, p = 4096, 2
    mesh = iga.Mesh(2, p, (n, n), (p + 1, p + 1), stream=stream)
    tune_us = [] if args.tile2d else mesh.autotune(iga.TUNE_APPLY, reps=5)
    if args.tile2d:
        for key, v in zip((iga.TILE_2D_STRIP, iga.TILE_2D_ROWS, iga.TILE_2D_ORDER), args.tile2d.split(",")):
            mesh.set_tile(key, int(v))
    g = torch.Generator(device="cuda")
    g.manual_seed(2)
    u0 = torch.randn((n + p, n + p), dtype=torch.float64, device="cuda", generator=g)
    sets = [(u0.clone(), torch.empty_like(u0), torch.empty_like(u0)) for _ in range(2)]
    steps = 40
    for k in range(2):
        u, m, l = sets[k % 2]
        mesh.apply(iga.PG, u, out_mass=m, out_lap=l)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        for k in range(steps):
            u, m, l = sets[k % 2]
            mesh.apply(iga.PG, u, out_mass=m, out_lap=l)
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    graph.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    per_s = e0.elapsed_time(e1) * 1e-3 / steps
    nbytes = 24 * u0.numel()
    out = {"workload": "2D, quadratic C1 B-splines, 4096x4096 elements, 3x3 Gauss, FP64, PG fused apply",
           "tile": mesh.tile(), "tile_candidates_us": [round(float(t), 3) for t in tune_us],
           "avg_launch_us": per_s * 1e6, "algorithmic_bytes_per_launch": nbytes,
           "achieved_GBs": nbytes / per_s / 1e9, "frac": nbytes / per_s / (HBM_PEAK_GBS * 1e9)}
    mesh.close()
    del sets, u0
    return out


def run_c2(args):
    import torch
    from paper_1910_08535_amd import iga, inputs

    c = inputs.Apply2D()
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    mesh = iga.Mesh(2, c.p, c.ne, c.nq, stream=stream)
    # the library's autotuner picks the tile (strip width, chunk rows, chunk order), unless
    # --tile2d fixes it (profiling runs: a profiler's own overhead can reorder the
    # candidates, so the profiled run is given the choice of the unprofiled one)
    tune_us = []
    if args.tile2d:
        for key, v in zip((iga.TILE_2D_STRIP, iga.TILE_2D_ROWS, iga.TILE_2D_ORDER), args.tile2d.split(",")):
            mesh.set_tile(key, int(v))
    else:
        tune_us = mesh.autotune(iga.TUNE_APPLY, reps=20)
    tile = mesh.tile()
    kernel = (f"iga::apply2d_kernel<2, {tile['rows']}, 3, true>" if tile["strip"] == 128
              else f"iga::apply2d1_kernel<2, {tile['rows']}, 3>")
    u0 = torch.from_numpy(c.coefs()).to("cuda")
    set_bytes = BYTES_C2
    nsets = max(1, -(-args.rotate_mb * 2**20 // set_bytes))
    sets = []
    for _ in range(nsets):
        sets.append((u0.clone(), torch.empty_like(u0), torch.empty_like(u0)))
    torch.cuda.synchronize()

    def step(k):
        u, m, l = sets[k % nsets]
        mesh.apply(iga.PG, u, out_mass=m, out_lap=l)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        for k in range(args.steps):
            step(k)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    graph.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    per_launch_s = gpu_ms * 1e-3 / args.steps

    # results of the timed launches against a fresh single launch (same kernel)
    u, m, l = sets[(args.steps - 1) % nsets]
    m2, l2 = mesh.apply(iga.PG, u)
    torch.cuda.synchronize()
    assert torch.equal(m, m2) and torch.equal(l, l2)

    # copy floor: the same bytes (one read, two streamed writes per coefficient) moved by a
    # plain copy kernel over the same rotated buffer sets, timed the same way
    n = u0.numel()

    def copy_step(k):
        u, m, l = sets[k % nsets]
        iga.iga_copy_probe(u.data_ptr(), m.data_ptr(), l.data_ptr(), n, stream.cuda_stream)

    for k in range(args.warmup):
        copy_step(k)
    cgraph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cgraph, stream=stream):
        for k in range(args.steps):
            copy_step(k)
    torch.cuda.synchronize()
    ev0.record(stream)
    cgraph.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    copy_s = ev0.elapsed_time(ev1) * 1e-3 / args.steps
    assert torch.equal(sets[0][1], sets[0][0]) and torch.equal(sets[0][2], sets[0][0])

    achieved = BYTES_C2 / per_launch_s / 1e9
    traffic = measured_traffic("apply2d_p2_1024", kernel)
    large = large_2d(args, stream)
    out = {
        "metric": "RHS Gauss-points/s (PG fused mass+Laplacian apply)",
        "value": GP_C2 * args.steps / wall,
        "unit": "GP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded N(0,1) coefficients)",
        "config": {"workload": "2D Laplace, quadratic C1 B-splines, 1024x1024 elements, "
                               "3x3 Gauss, FP64, PG fused apply (mass + Laplacian rows), "
                               "support spans",
                   "elements": [1024, 1024], "p": 2, "nq": [3, 3],
                   "gauss_points_per_step": GP_C2, "buffer_sets": nsets,
                   "rotated_bytes": nsets * set_bytes},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": kernel, "tile": tile, "tile_source": "fixed" if args.tile2d else "autotuned",
                     "tile_candidates_us": [round(float(t), 3) for t in tune_us],
                     "algorithmic_bytes_per_launch": BYTES_C2,
                     "avg_launch_us": per_launch_s * 1e6},
        "large_2d": large,
        "copy_floor": {"kernel": "iga::copy2_kernel (read once, two streamed writes)",
                       "avg_launch_us": copy_s * 1e6, "GBs": BYTES_C2 / copy_s / 1e9,
                       "frac": BYTES_C2 / copy_s / 1e9 / HBM_PEAK_GBS,
                       "apply_over_floor": per_launch_s / copy_s},
    }
    return out


def run_c3(args) -> dict:
    """3D heat u_t = Lap u + f, cubic C2 B-splines, 128^3 elements, 4^3 Gauss, dt = 1e-6,
    f = sin sin sin: 100 explicit PG steps (one cached HIP graph of 100 step launches),
    timed with HIP events on the mesh's stream.  The 36 MB working set (u and the step's
    work buffer) stays in the 256 MB Infinity Cache across steps, as in the application;
    a second figure steps 16 independent problems round-robin (576 MB) so that every
    step reads and writes HBM."""
    import torch
    from paper_1910_08535_amd import iga, inputs

    c = inputs.Heat3D()
    ncoef = 1
    for n in c.ne:
        ncoef *= n + c.p
    gp_step = c.ne[0] * c.ne[1] * c.ne[2] * (c.p + 1) ** 3
    bytes_step = 16 * ncoef
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    mesh = iga.Mesh(3, c.p, c.ne, c.nq, stream=stream)
    # the library's autotuner picks the tile (z-chunk planes, tile rows and columns), unless
    # --tile3d fixes it; the 16 meshes of the rotated run below take the same setting
    tune_us = []
    if args.tile3d:
        tkeys = (iga.TILE_3D_PLANES, iga.TILE_3D_ROWS, iga.TILE_3D_COLS)
        tvals = [int(v) for v in args.tile3d.split(",")]
        for key, v in zip(tkeys, tvals):
            mesh.set_tile(key, v)
    else:
        tune_us = mesh.autotune(iga.TUNE_STEP, reps=20)
    tile = mesh.tile()
    u0 = torch.from_numpy(c.coefs()).to("cuda")
    u = u0.clone()
    for _ in range(2):   # the second identical call captures the graph
        mesh.explicit_step(u, c.dt, sin_amp=c.sin_amp, nsteps=c.nsteps)
    torch.cuda.synchronize()
    reps = max(1, args.c3_reps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        mesh.explicit_step(u, c.dt, sin_amp=c.sin_amp, nsteps=c.nsteps)
    e1.record(stream)
    torch.cuda.synchronize()
    step_s = e0.elapsed_time(e1) * 1e-3 / (reps * c.nsteps)
    # 16 independent problems, two steps each in turn (each call replays the problem's
    # own cached 2-step graph; u and the work buffer ping-pong, no copy)
    nprob = 16
    meshes = [iga.Mesh(3, c.p, c.ne, c.nq, stream=stream) for _ in range(nprob)]
    if args.tile3d:
        for m in meshes:
            for key, v in zip(tkeys, tvals):
                m.set_tile(key, v)
    us = [u0.clone() for _ in range(nprob)]
    for _ in range(2):
        for m, x in zip(meshes, us):
            m.explicit_step(x, c.dt, sin_amp=c.sin_amp, nsteps=2)
    torch.cuda.synchronize()
    rounds = 4
    e0.record(stream)
    for _ in range(rounds):
        for m, x in zip(meshes, us):
            m.explicit_step(x, c.dt, sin_amp=c.sin_amp, nsteps=2)
    e1.record(stream)
    torch.cuda.synchronize()
    rot_s = e0.elapsed_time(e1) * 1e-3 / (rounds * nprob * 2)
    for m in meshes:
        m.close()
    mesh.close()
    # sum-factorized work per output row: z pass 2 x (2p+1) FMA, y and x passes 3 x (2p+1)
    flops_step = 2 * 8 * (2 * c.p + 1) * ncoef
    return {"workload": "3D heat, cubic C2 B-splines, 128^3 elements, 4^3 Gauss, FP64, dt = 1e-6, "
                        "100 explicit PG steps (lumped), f = sin(pi x) sin(pi y) sin(pi z)",
            "gauss_points_per_step": gp_step, "algorithmic_bytes_per_step": bytes_step,
            "us_per_step": step_s * 1e6, "GPs": gp_step / step_s,
            "mall_resident_frac_of_hbm_peak": bytes_step / step_s / (HBM_PEAK_GBS * 1e9),
            "algorithmic_flop_per_step": flops_step,
            "fp64_frac": flops_step / step_s / (FP64_PEAK_TFLOPS * 1e12),
            "note": "us_per_step: working set in the Infinity Cache across steps, as in the "
                    "application; roofline: 16 problems stepped in turn, every step from HBM",
            "rotated_16_problems": {"us_per_step": rot_s * 1e6, "GPs": gp_step / rot_s,
                                    "hbm_frac": bytes_step / rot_s / (HBM_PEAK_GBS * 1e9)},
            "roofline": {"bound": "hbm", "achieved": bytes_step / rot_s / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": bytes_step / rot_s / (HBM_PEAK_GBS * 1e9),
                         "traffic": measured_traffic("heat3d_p3_128"),
                         "kernel": "iga::apply3d_kernel<3, 9>", "tile": tile,
                         "tile_source": "fixed" if args.tile3d else "autotuned",
                         "tile_candidates_us": [round(float(t), 3) for t in tune_us],
                         "algorithmic_bytes_per_launch": bytes_step, "avg_launch_us": rot_s * 1e6}}


def run_c4(args) -> dict:
    """256 independent 2D problems (p in {2,3}, n, m uniform in [32, 1024], seed 4), each a
    fused PG apply.  Plain: one kernel launch per problem (the 256 launches replayed as one
    HIP graph, so launch overhead is minimal); batched: one persistent launch over all
    problems (iga_batch, autotuned chunk height).  Inputs resident in HBM (~1.8 GB).
    Device times come from HIP events on the launching stream."""
    import torch
    from paper_1910_08535_amd import iga, inputs

    jobs, coefs = inputs.batch_jobs()
    stream = torch.cuda.Stream()   # graph capture needs a non-default stream
    torch.cuda.set_stream(stream)
    dev = []
    gp = 0
    nbytes = 0
    for j, u in zip(jobs, coefs):
        ud = torch.from_numpy(u).cuda()
        dev.append((j.p, j.ne, ud, torch.empty_like(ud), torch.empty_like(ud)))
        gp += j.ne[0] * j.ne[1] * (j.p + 1) ** 2
        nbytes += 24 * ud.numel()
    torch.cuda.synchronize()
    # batched: the autotuner times `reps` persistent launches per chunk height
    b = iga.Batch(max_jobs=len(dev), stream=stream)
    b.submit(dev)
    best_rows, batch_ms = b.autotune(reps=args.batch_reps)
    b.flush()
    b.wait()
    # host-inclusive rounds: submit + flush of all 256 jobs each round
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_reps):
        b.submit(dev)
        b.flush()
    b.wait()
    round_s = (time.perf_counter() - t0) / args.batch_reps
    b.close()
    # plain: one launch per problem (the library's default 2D tile), 256 launches in one
    # graph
    meshes = [iga.Mesh(2, p, ne, (p + 1, p + 1), stream=stream) for p, ne, *_ in dev]
    for m, (p, ne, u, mo, lo) in zip(meshes, dev):
        m.apply(iga.PG, u, out_mass=mo, out_lap=lo)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        for m, (p, ne, u, mo, lo) in zip(meshes, dev):
            m.apply(iga.PG, u, out_mass=mo, out_lap=lo)
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.batch_reps):
        graph.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / args.batch_reps
    batch_s, plain_s = batch_ms * 1e-3, plain_ms * 1e-3
    return {"workload": "256 independent 2D problems, p in {2,3}, n,m ~ U[32,1024] (seed 4), "
                        "fused PG apply each",
            "gauss_points": gp, "algorithmic_bytes": nbytes, "chunk_rows": best_rows,
            "batched_GPs": gp / batch_s, "plain_GPs": gp / plain_s,
            "batched_ms": batch_ms, "plain_ms": plain_ms, "speedup": plain_s / batch_s,
            "batched_hbm_frac": nbytes / batch_s / (HBM_PEAK_GBS * 1e9),
            "plain_hbm_frac": nbytes / plain_s / (HBM_PEAK_GBS * 1e9),
            "batched_round_ms_host_inclusive": round_s * 1e3}


def run_ads(args) -> dict:
    """Galerkin L2 projection with the alternating-directions direct solve, at the size of
    the paper's projection table (3D, 256^3 elements, p = 2 and 3, (p+1)^3 Gauss points):
    right-hand side b_r = int B_r f with f = sin(pi x) sin(pi y) sin(pi z), then
    (M_z (x) M_y (x) M_x) u = b in three families of 1D banded solves (factors computed
    once per mesh, outside the timed region).  Also one consistent-mass Galerkin Euler step
    of the 3D heat workload (128^3, p = 3; the step is unstable at dt = 1e-6, so only its
    time is reported), and the refined-test-space PG projection (256^3, p = 2, refine 4):
    the sine rows and the solve with the LU factors of its square PG mass.  The solve of
    families with few lines, partitioned into chunks, at 2D 1024^2 and 1D 10^6 elements
    (p = 2; b = N(0,1), seed 21).  Every call is timed with HIP events on the mesh's
    stream over `reps` calls after two warm-up calls.  Algorithmic HBM bytes of a solve:
    each family reads and writes every coefficient once, 16 B per coefficient and axis."""
    import torch
    from paper_1910_08535_amd import iga

    reps = max(1, args.ads_reps)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    out = {}
    for p in (2, 3):
        ne = (256, 256, 256)
        mesh = iga.Mesh(3, p, ne, (p + 1,) * 3, stream=stream)
        b = torch.empty(mesh.coef_shape(), dtype=torch.float64, device="cuda")
        u = torch.empty_like(b)
        n = b.numel()
        t_rhs = timed(lambda: mesh.rhs(iga.GALERKIN_BYPARTS, None, 0.0, 0.0, 1.0, sin_amp=1.0, out=b))
        t_solve = timed(lambda: mesh.solve(b, out=u))
        out[f"projection_256_p{p}"] = {
            "dofs": n, "us_rhs": t_rhs * 1e6, "us_solve": t_solve * 1e6,
            "us_projection": (t_rhs + t_solve) * 1e6,
            "dofs_per_s_solve": n / t_solve,
            "solve_hbm_frac": 48.0 * n / t_solve / (HBM_PEAK_GBS * 1e9)}
        mesh.close()
        del b, u
    # the refined-test-space PG projection (refine 4, regular square system): rows of the
    # sine source, then the solve with the LU factors of the PG mass
    for p in (2,):
        ne = (256, 256, 256)
        mesh = iga.Mesh(3, p, ne, (p + 1,) * 3, stream=stream, spans="refined", refine=(4, 4, 4))
        b = torch.empty(mesh.coef_shape(), dtype=torch.float64, device="cuda")
        u = torch.empty_like(b)
        n = b.numel()
        t_rhs = timed(lambda: mesh.rhs(iga.PG, None, 0.0, 0.0, 1.0, sin_amp=1.0, out=b))
        t_solve = timed(lambda: mesh.solve(b, form=iga.PG, out=u))
        out[f"refined_pg_projection_256_p{p}"] = {
            "dofs": n, "refine": 4, "us_rhs": t_rhs * 1e6, "us_solve": t_solve * 1e6,
            "dofs_per_s_solve": n / t_solve,
            "solve_hbm_frac": 48.0 * n / t_solve / (HBM_PEAK_GBS * 1e9)}
        mesh.close()
        del b, u
    # families with few lines: the partitioned solve
    for dim, ne in ((2, (1024, 1024)), (1, (1000000,))):
        mesh = iga.Mesh(dim, 2, ne, (3,) * dim, stream=stream)
        g = torch.Generator(device="cuda").manual_seed(21)
        b = torch.randn(mesh.coef_shape(), dtype=torch.float64, device="cuda", generator=g)
        u = torch.empty_like(b)
        n = b.numel()
        t_solve = timed(lambda: mesh.solve(b, out=u))
        key = f"solve_{dim}d_{ne[0]}_p2"
        out[key] = {"dofs": n, "us_solve": t_solve * 1e6, "dofs_per_s_solve": n / t_solve,
                    "solve_hbm_frac": 16.0 * dim * n / t_solve / (HBM_PEAK_GBS * 1e9)}
        mesh.close()
        del b, u
    mesh = iga.Mesh(3, 3, (128, 128, 128), (4, 4, 4), stream=stream)
    u = torch.zeros(mesh.coef_shape(), dtype=torch.float64, device="cuda")
    t_step = timed(lambda: mesh.galerkin_step(u, 1e-6, iga.GALERKIN_LAPLACIAN, sin_amp=1.0))
    out["galerkin_step_128_p3"] = {"us_per_step": t_step * 1e6,
                                   "GPs": 128 ** 3 * 64 / t_step}
    mesh.close()
    out["kernel"] = ("iga::ads_seg_kernel<P> (one launch per axis); families with few lines: "
                     "chunk solves, then iga::part_fix_kernel (block-diagonal reduced system and "
                     "correction) or the reduced sweeps and iga::part_correct_kernel")
    return out


def run_laplace(args) -> dict:
    """The Laplace problem with mixed conditions in the PG form (quadratic C1, 3x3 Gauss,
    unit square): -Lap u = f with f given at the Gauss points, u = 0 on x = 0 and
    du/dn = G on the other sides (a table of Gauss-point values on x = 1, a constant on
    y = 0, 1).  Times, per size, the right-hand side (domain rows, Neumann rows, Dirichlet
    rows) and the operator application to u (Laplacian rows, flux rows, identity rows),
    each sequence captured 20 times into a HIP graph and replayed (device time; the eager
    calls, whose small launches are bound by the host's launch rate, are reported
    beside).  HIP events on the mesh's stream.  The sizes are the largest of the paper's
    2D Laplace table (256^2) and the headline 1024^2."""
    import numpy as np
    import torch
    from paper_1910_08535_amd import iga, inputs

    reps = max(1, args.ads_reps)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    out = {}
    for n in (256, 1024):
        mesh = iga.Mesh(2, 2, (n, n), (3, 3), stream=stream)
        u = torch.from_numpy(inputs.normal_coefs((n, n), 2, 6)).cuda()
        f = torch.from_numpy(inputs.uniform_table((3 * n, 3 * n), 7)).cuda()
        g = torch.from_numpy(inputs.uniform_table((3 * n,), 8)).cuda()
        neu = [(1, g, 0.0), (2, None, 0.5), (3, None, -0.5)]
        b = torch.empty(mesh.shape(iga.PG), dtype=torch.float64, device="cuda")
        au = torch.empty_like(b)

        def rhs():
            mesh.rhs(iga.PG, None, 0.0, 0.0, 1.0, f_table=f, out=b)
            mesh.boundary_terms(iga.PG, neu, b, beta=1.0)
            mesh.dirichlet_rows(iga.PG, 0b0001, b)

        def apply():
            mesh.apply(iga.PG, u, mass=False, out_lap=au)
            au.neg_()
            mesh.boundary_terms(iga.PG, neu, au, u=u, alpha=1.0)
            mesh.dirichlet_rows(iga.PG, 0b0001, au, u=u)

        t_rhs, t_apply = timed(rhs), timed(apply)
        b_ref, au_ref = b.clone(), au.clone()

        def graphed(fn, k=20):
            # k calls captured once (scratch already sized by the calls above), replayed
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream):
                for _ in range(k):
                    fn()
            graph.replay()
            torch.cuda.synchronize()
            e0.record(stream)
            graph.replay()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) * 1e-3 / k

        g_rhs, g_apply = graphed(rhs), graphed(apply)
        # every replay recomputes the same rows as the eager calls
        assert torch.equal(b, b_ref) and torch.equal(au, au_ref)
        out[f"n{n}"] = {"dofs": (n + 2) ** 2, "us_rhs": g_rhs * 1e6, "us_apply": g_apply * 1e6,
                        "GPs_rhs": 9 * n * n / g_rhs,
                        "us_rhs_eager": t_rhs * 1e6, "us_apply_eager": t_apply * 1e6}
        mesh.close()
    return out


def run_reduced(args) -> dict:
    """Reduced quadrature in the PG form (Section 4.1): the 2-point Gauss rule on every axis
    against the (p+1)-point rule.  The rows of the u terms come from band factors built
    at set-up, whatever the rule, so per call the rule changes only what a source given
    at the Gauss points costs: its table holds 2^d instead of (p+1)^d values per element.
    Times rhs(PG, u, alpha = beta = gamma = 1, f_table) per rule for 2D 1024^2, p = 2 and
    3D 128^3, p = 3, HIP events on the mesh's stream; the tables (seeded uniform values
    in [-1, 1)) are used in turn, enough of them to exceed 600 MB, so each call reads its
    table from HBM.  Algorithmic bytes: the table, u and the output rows.  Beside it, the
    source rows alone (gamma = 1, no u) in the PG form and, with the (p+1)-point rule, in
    the Galerkin form (test functions evaluated at every Gauss point): the generation
    cost of the two methods on the same table (Table 1's comparison)."""
    import math
    import torch
    from paper_1910_08535_amd import iga, inputs

    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for dim, p, n in ((2, 2, 1024), (3, 3, 128)):
        ne = (n,) * dim
        case = {}
        for nq in (p + 1, 2):
            mesh = iga.Mesh(dim, p, ne, (nq,) * dim, stream=stream)
            u = torch.from_numpy(inputs.normal_coefs(ne, p, 6)).cuda()
            shape = inputs.gauss_shape(ne, (nq,) * dim)
            tbytes = math.prod(shape) * 8
            gen = torch.Generator(device="cuda")
            gen.manual_seed(7)
            tabs = [torch.empty(shape, dtype=torch.float64, device="cuda").uniform_(-1.0, 1.0, generator=gen)
                    for _ in range(max(1, math.ceil(600e6 / tbytes)))]
            reps = max(10, len(tabs))

            def timed(form, uu, alpha, beta):
                b = torch.empty(mesh.shape(form), dtype=torch.float64, device="cuda")
                for t in tabs[:2]:
                    mesh.rhs(form, uu, alpha, beta, 1.0, f_table=t, out=b)
                torch.cuda.synchronize()
                e0.record(stream)
                for i in range(reps):
                    mesh.rhs(form, uu, alpha, beta, 1.0, f_table=tabs[i % len(tabs)], out=b)
                e1.record(stream)
                torch.cuda.synchronize()
                return e0.elapsed_time(e1) * 1e3 / reps, b.numel()

            us, nrow = timed(iga.PG, u, 1.0, 1.0)
            nbytes = tbytes + u.numel() * 8 + nrow * 8
            rec = {"us_rhs": us, "table_bytes": tbytes, "algorithmic_bytes": nbytes,
                   "GBs": nbytes / us * 1e-3, "hbm_frac": nbytes / us * 1e-3 / 8000.0,
                   "us_source_only": timed(iga.PG, None, 0.0, 0.0)[0]}
            if nq == p + 1:
                rec["us_source_only_galerkin"] = timed(iga.GALERKIN_BYPARTS, None, 0.0, 0.0)[0]
                rec["galerkin_over_pg_source"] = rec["us_source_only_galerkin"] / rec["us_source_only"]
            case[f"nq{nq}"] = rec
            del tabs
            mesh.close()
        case["speedup_2pt"] = case[f"nq{p + 1}"]["us_rhs"] / case["nq2"]["us_rhs"]
        out[f"{dim}d_{n}_p{p}"] = case
    return out


def stage_requests(reqs) -> int:
    """Puts every request's coefficients (seeded N(0,1), as the request's seed draws them)
    and, for RHS requests, its two output arrays on the device, so that the timed serving
    runs start with inputs in HBM."""
    import torch
    gen = torch.Generator(device="cuda")
    total = 0
    for r in reqs:
        gen.manual_seed(r.seed)
        shape = tuple(n + r.p for n in reversed(r.ne))
        r.u = torch.randn(shape, dtype=torch.float64, device="cuda", generator=gen)
        r.out = torch.empty((2,) + shape, dtype=torch.float64, device="cuda") if r.kind == "rhs" else None
        total += r.u.numel() * 8 * (3 if r.kind == "rhs" else 1)
    torch.cuda.synchronize()
    return total


def run_c5(args) -> dict:
    """Serving: a seeded Poisson stream (2000 req/s) of RHS / explicit-step requests, 1D (up
    to 1e6 elements), 2D (up to 2048^2), 3D (up to 192^3), p in {2,3}, 200 GB admission
    budget, request coefficients already in HBM.  (a) arrivals in real time: p50/p99
    latency; (b) every request present at t = 0: served throughput; (c) the same requests
    one at a time, each waited for before the next (plain)."""
    import torch
    from paper_1910_08535_amd import iga, inputs, serve

    reqs = inputs.request_stream(rate=2000.0, seconds=args.serve_seconds, seed=5)
    staged = stage_requests(reqs)
    srv = serve.Server(budget_bytes=200 * 10**9)
    realtime = srv.run(reqs)
    srv.close()
    stage_requests(reqs)
    srv = serve.Server(budget_bytes=200 * 10**9)
    saturated = srv.run(reqs, time_scale=0.0)
    srv.close()
    # plain: one request at a time, each waited for before the next (meshes cached)
    stage_requests(reqs)
    meshes = serve.MeshCache([torch.cuda.current_stream()])   # the server's cache policy
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gp = 0
    for r in reqs:
        mesh = meshes.get(r.dim, r.p, r.ne)
        if r.kind == "rhs":
            mesh.apply(iga.PG, r.u, out_mass=r.out[0], out_lap=r.out[1])
        else:
            h = min(1.0 / n for n in r.ne)
            mesh.explicit_step(r.u, h * h / 64.0, sin_amp=1.0, nsteps=r.nsteps)
        torch.cuda.synchronize()
        gp += serve.request_work(r)[0]
    plain_s = time.perf_counter() - t0
    meshes.close()
    for r in reqs:
        r.u = r.out = None
    return {"workload": f"Poisson 2000 req/s for {args.serve_seconds} s (seed 5): RHS / explicit "
                        "step, 1D <= 1e6, 2D <= 2048^2, 3D <= 192^3 elements, p in {2,3}, "
                        "200 GB budget, request coefficients staged in HBM",
            "requests": len(reqs), "staged_bytes": staged, "realtime": realtime,
            "saturated": saturated, "plain_GPs": gp / plain_s, "plain_s": plain_s,
            "served_vs_plain": saturated["GPs"] / (gp / plain_s)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--rotate-mb", type=int, default=600,
                    help="distinct buffer bytes cycled through (defeats the Infinity Cache)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-others", action="store_true",
                    help="time the oracle on the C2 workload only")
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-problem batched leg")
    ap.add_argument("--batch-reps", type=int, default=10)
    ap.add_argument("--no-heat3d", action="store_true", help="skip the 3D explicit-step leg")
    ap.add_argument("--c3-reps", type=int, default=5, help="100-step runs timed in the 3D leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-ads", action="store_true", help="skip the Galerkin projection/solve leg")
    ap.add_argument("--ads-reps", type=int, default=10)
    ap.add_argument("--no-laplace", action="store_true", help="skip the mixed Laplace leg")
    ap.add_argument("--no-reduced", action="store_true",
                    help="skip the 2-point against (p+1)-point PG right-hand-side leg")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--tile2d", default="",
                    help="STRIP,ROWS,ORDER: fix the 2D tile instead of autotuning it")
    ap.add_argument("--tile3d", default="",
                    help="PLANES,ROWS,COLS: fix the 3D tile instead of autotuning it")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run a plain copy of this many MiB first (counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the path runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.copy_probe_mb > 0:
        copy_probe(args.copy_probe_mb)
    out = run_c2(args)
    if not args.no_heat3d:
        out["heat3d"] = run_c3(args)
    if not args.no_ads:
        out["ads"] = run_ads(args)
    if not args.no_laplace:
        out["laplace2d"] = run_laplace(args)
    if not args.no_reduced:
        out["reduced_quadrature"] = run_reduced(args)
    if not args.no_batched:
        out["batched"] = run_c4(args)
    if not args.no_serving:
        out["serving"] = run_c5(args)
    if rank == 0 and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
