"""Serving: a mixed request stream (1D/2D/3D, RHS and explicit steps) through the
continuous-batching server gives every request the same result as running it alone
(bit for bit: same kernels, same launch geometry), matches the oracle, and keeps the
admitted device memory inside the budget."""
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
    """Explicit-step requests leave their work buffer with the cached context: the cache
    counts it, so many distinct step shapes under a small cache limit keep the cached
    device memory bounded (the least recently used contexts are evicted)."""
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
        ne = (76 + k, 77, 78 + (k % 3))   # distinct shapes, about 4 MB of coefficients each
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
