"""Serving: a mixed request stream (1D/2D/3D, RHS and explicit steps) through the
continuous-batching server gives every request the same result as running it alone on a
context (bit for bit), matches the oracle, and keeps the admitted device memory inside the
budget.  Requests whose axes all have at least 3p+1 elements advance in batched
iterations (one step per iteration); the others run on cached contexts."""
import numpy as np
import pytest

from paper_1910_08535_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_1910_08535_amd import iga, serve
    assert torch.cuda.is_available()
    iga.lib()
    return iga, serve


def _alone(iga, req):
    import torch
    shape = tuple(n + req.p for n in reversed(req.ne))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(req.seed)
    u = torch.randn(shape, dtype=torch.float64, device="cuda", generator=gen)
    mesh = iga.Mesh(req.dim, req.p, req.ne, (req.p + 1,) * req.dim)
    if req.kind == "rhs":
        m, l = mesh.apply(iga.PG, u)
        out = (u, m, l)
    else:
        h = min(1.0 / n for n in req.ne)
        for _ in range(req.nsteps):
            mesh.explicit_step(u, h * h / 64.0, sin_amp=1.0, nsteps=1)
        out = (u,)
    torch.cuda.synchronize()
    return out


def test_mix_equals_alone_and_oracle(mods, orc):
    import torch
    iga, serve = mods
    reqs = inputs.request_stream(rate=600.0, seconds=0.1, seed=21, max_1d=20000, max_2d=160,
                                 max_3d=20)
    assert len(reqs) > 30 and {r.dim for r in reqs} == {1, 2, 3}
    assert {r.kind for r in reqs} == {"rhs", "step"}
    # requests with an axis below 3p+1 elements: served on contexts, not batched
    t = reqs[-1].t_arrive
    small = [inputs.Request(t, "rhs", 3, 2, (5, 9, 8), 0, 11), inputs.Request(t, "step", 2, 3, (40, 6), 3, 12),
             inputs.Request(t, "step", 1, 2, (6,), 2, 13), inputs.Request(t, "rhs", 2, 2, (4, 33), 0, 14)]
    assert not any(serve.batched(r) for r in small) and all(serve.batched(r) for r in reqs)
    reqs = reqs + small
    srv = serve.Server(budget_bytes=64 << 20, streams=3, keep_outputs=True)
    stats = srv.run(reqs)
    torch.cuda.synchronize()
    assert stats["requests"] == len(reqs) and stats["p99_ms"] >= stats["p50_ms"] > 0
    assert srv.used == 0
    launches = {r.batch_launch for r in srv.done if r.batch_launch >= 0}
    assert len(launches) >= 1
    for rec in srv.done:
        ref = _alone(iga, rec.req)
        for got, want in zip(rec.tensors[1:] or rec.tensors, ref[1:] or ref):
            assert torch.equal(got, want), rec.req
    # a few against the oracle
    checked = 0
    for rec in srv.done:
        r = rec.req
        if r.kind != "rhs" or np.prod(r.ne) > 4000:
            continue
        pb = orc.Problem(dim=r.dim, p=r.p, ne=r.ne, nq=(r.p + 1,) * r.dim)
        u = rec.tensors[0].cpu().numpy()
        ref = orc.rhs(pb, orc.PG, u, beta=1.0)
        err = np.abs(rec.tensors[2].cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err <= 1e-12
        checked += 1
    assert checked >= 3
    srv.close()


def test_budget_limits_admission(mods):
    iga, serve = mods
    reqs = inputs.request_stream(rate=2000.0, seconds=0.02, seed=3, max_1d=5000, max_2d=96,
                                 max_3d=16)
    budget = max(serve.footprint(r) for r in reqs)   # one request at a time
    srv = serve.Server(budget_bytes=budget, streams=2)
    srv.run(reqs)
    assert len(srv.done) == len(reqs)
    assert 0 < srv.peak <= budget and srv.used == 0
    srv.close()


def test_server_rejects_bad_requests(mods):
    import torch
    iga, serve = mods
    s = iga.NativeServer(nstreams=1, budget_bytes=1 << 20)
    u = torch.zeros(40, dtype=torch.float64, device="cuda")
    m, l = torch.empty_like(u), torch.empty_like(u)
    good = np.zeros(1, dtype=s.dtype)
    good["kind"], good["dim"], good["p"] = iga.REQ_RHS, 1, 2
    good["ne"][0] = [38, 1, 1]
    good["u"], good["mass_out"], good["lap_out"] = u.data_ptr(), m.data_ptr(), l.data_ptr()
    for field, value, code in (("p", 4, iga.IGA_E_UNSUPPORTED), ("dim", 0, iga.IGA_E_UNSUPPORTED),
                               ("kind", 7, iga.IGA_E_INVAL), ("lap_out", 0, iga.IGA_E_INVAL)):
        bad = good.copy()
        bad[field] = value
        with pytest.raises(iga.IGAError) as e:
            s.submit(bad)
        assert e.value.code == code, field
    big = good.copy()
    big["ne"][0] = [100000, 1, 1]   # more bytes than the whole budget
    with pytest.raises(iga.IGAError) as e:
        s.submit(big)
    assert e.value.code == iga.IGA_E_NOMEM
    t = s.submit(good)
    while True:
        done = s.progress()[0]
        if len(done):
            break
    assert done.tolist() == t.tolist() and s.stats()[0] == 0
    s.close()


def test_cache_counts_step_scratch(mods):
    """Explicit-step requests served on contexts leave their work buffer with the cached
    context: the cache counts it, so many distinct step shapes under a small cache limit
    keep the cached device memory bounded (the least recently used contexts are
    evicted)."""
    import torch
    iga, serve = mods
    limit = 8 << 20
    count = 40
    s = iga.NativeServer(nstreams=2, budget_bytes=1 << 30, cache_bytes=limit)
    bufs = []
    largest = 0
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for k in range(count):
        ne = (76 + k, 770, 6)   # distinct shapes, about 4 MB of coefficients each; z below
                                # 3p+1 elements, so they run on contexts
        u = torch.zeros(tuple(n + 2 for n in reversed(ne)), dtype=torch.float64, device="cuda")
        rec = np.zeros(1, dtype=s.dtype)
        rec["kind"], rec["dim"], rec["p"], rec["nsteps"] = iga.REQ_STEP, 3, 2, 2
        rec["ne"][0] = list(ne)
        rec["dt"], rec["sin_amp"], rec["u"] = 1e-6, 1.0, u.data_ptr()
        s.submit(rec)
        bufs.append(u)
        largest = max(largest, 2 * u.numel() * 8)
        cached, n = s.cache_stats()
        # the work buffer of each context is counted; at most the limit plus the newest
        assert cached <= limit + largest, (k, cached)
    while s.stats()[0] > 0:
        s.progress()
    cached, n = s.cache_stats()
    assert cached <= limit + largest and 1 <= n <= 4, (cached, n)
    torch.cuda.synchronize()
    # device memory held beyond the request buffers stays near the cache limit (the
    # stream-ordered pool keeps freed memory for reuse): far below one work buffer per shape
    held = free0 - torch.cuda.mem_get_info()[0] - sum(b.numel() * 8 for b in bufs)
    assert held < count * largest // 4, (held, largest)
    s.close()


def _native_rec(iga, s, kind, dim, p, ne, u, outs=None, nsteps=0, dt=0.0, amp=0.0):
    rec = np.zeros(1, dtype=s.dtype)
    rec["kind"], rec["dim"], rec["p"] = kind, dim, p
    rec["ne"][0] = list(ne) + [1] * (3 - dim)
    rec["u"] = u.data_ptr()
    if outs is not None:
        rec["mass_out"], rec["lap_out"] = outs[0].data_ptr(), outs[1].data_ptr()
    rec["nsteps"], rec["dt"], rec["sin_amp"] = nsteps, dt, amp
    return rec


def test_step_iterations_advance_together(mods):
    """Step requests submitted together advance one step per iteration: the number of
    iterations is the largest step count, whatever the mix of dimensions, and each result
    (with and without a source, odd and even step counts) equals the same steps run alone
    on a context.  No context is created for them."""
    import torch
    iga, serve = mods
    cases = [(1, 2, (700,), 3, 1.0), (1, 3, (901,), 4, 0.0), (2, 2, (40, 33), 5, 1.0), (2, 3, (31, 64), 2, 0.0),
             (3, 2, (12, 9, 10), 7, 1.0), (3, 3, (10, 11, 13), 6, 0.0), (2, 2, (129, 18), 1, 1.0)]
    s = iga.NativeServer(nstreams=2, budget_bytes=1 << 30)
    gen = torch.Generator(device="cuda")
    us, refs = [], []
    recs = []
    for k, (dim, p, ne, n, amp) in enumerate(cases):
        gen.manual_seed(100 + k)
        u = torch.randn(tuple(m + p for m in reversed(ne)), dtype=torch.float64, device="cuda", generator=gen)
        dt = min(1.0 / m for m in ne) ** 2 / 64.0
        ref = u.clone()
        mesh = iga.Mesh(dim, p, ne, (p + 1,) * dim)
        for _ in range(n):
            mesh.explicit_step(ref, dt, sin_amp=amp, nsteps=1)
        torch.cuda.synchronize()
        mesh.close()
        us.append(u)
        refs.append(ref)
        recs.append(_native_rec(iga, s, iga.REQ_STEP, dim, p, ne, u, nsteps=n, dt=dt, amp=amp))
    torch.cuda.synchronize()
    s.submit(np.concatenate(recs))
    got = 0
    while got < len(cases):
        got += len(s.progress()[0])
    assert s.stats()[2] == max(c[3] for c in cases)
    assert s.cache_stats()[1] == 0
    torch.cuda.synchronize()
    for (dim, p, ne, n, amp), u, ref in zip(cases, us, refs):
        assert torch.equal(u, ref), (dim, p, ne, n, amp)
    assert s.stats()[0] == 0
    s.close()


def test_batched_memory_returns(mods):
    """The tables and work buffers of batched jobs go back to the device once the jobs
    are done: repeated rounds of many batched requests hold no growing device memory, and
    the admitted bytes return to zero."""
    import torch
    iga, serve = mods
    reqs = inputs.request_stream(rate=4000.0, seconds=0.02, seed=8, max_1d=30000, max_2d=200, max_3d=24)
    assert all(serve.batched(r) for r in reqs)
    srv = serve.Server(budget_bytes=1 << 30, streams=2)
    srv.run(reqs, time_scale=0.0)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        for r in reqs:
            r.u = r.out = None
        srv.run(reqs, time_scale=0.0)
        torch.cuda.synchronize()
    assert srv.used == 0 and srv.native.cache_stats()[1] == 0
    assert torch.cuda.mem_get_info()[0] >= free1 - (64 << 20)
    srv.close()
