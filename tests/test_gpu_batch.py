"""Batched execution (one persistent launch over many independent 2D problems):
results equal iga_apply bit for bit (same kernel code, same tile setting), match the
oracle, and the queue honours its capacity, memory budget and job states."""
import numpy as np
import pytest

from paper_1910_08535_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def iga():
    import torch
    from paper_1910_08535_amd import iga as m
    assert torch.cuda.is_available()
    m.lib()
    return m


def _jobs(count, seed, lo=1, hi=300):
    import torch
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        p = int(rng.integers(2, 4))
        nx, ny = int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))
        u = torch.from_numpy(rng.standard_normal((ny + p, nx + p))).cuda()
        out.append((p, (nx, ny), u, torch.full_like(u, np.nan), torch.full_like(u, np.nan)))
    return out


def _reference(iga, p, ne, u, rows):
    mesh = iga.Mesh(2, p, ne, (p + 1, p + 1))
    mesh.set_tile(iga.TILE_2D_ROWS, rows)
    return mesh.apply(iga.PG, u)


def test_batch_equals_single_launches_bitwise(iga):
    import torch
    jobs = _jobs(40, seed=1) + [(2, (1, 1), torch.randn(3, 3, dtype=torch.float64).cuda(), None, None)]
    jobs[-1] = (jobs[-1][0], jobs[-1][1], jobs[-1][2], torch.empty_like(jobs[-1][2]),
                torch.empty_like(jobs[-1][2]))
    b = iga.Batch(max_jobs=64)
    tickets = b.submit(jobs)
    assert all(b.poll(t) == iga.JOB_QUEUED for t in tickets)
    b.flush()
    b.wait()
    assert all(b.poll(t) == iga.JOB_DONE for t in tickets)
    for p, ne, u, m, l in jobs:
        rm, rl = _reference(iga, p, ne, u, 8)
        torch.cuda.synchronize()
        assert torch.equal(m, rm) and torch.equal(l, rl), (p, ne)
    b.close()


def test_batch_matches_oracle(iga, orc):
    import torch
    jobs = _jobs(6, seed=2, lo=1, hi=150)
    b = iga.Batch()
    b.submit(jobs)
    b.flush()
    b.wait()
    for p, ne, u, m, l in jobs:
        pb = orc.Problem(dim=2, p=p, ne=ne, nq=(p + 1, p + 1))
        un = u.cpu().numpy()
        for got, kw in ((m, dict(alpha=1.0)), (l, dict(beta=1.0))):
            ref = orc.rhs(pb, orc.PG, un, **kw)
            err = np.abs(got.cpu().numpy() - ref).max() / np.abs(ref).max()
            assert err <= TOL, (p, ne, err)
    b.close()


def test_autotune_keeps_results(iga):
    import torch
    jobs = _jobs(12, seed=3, lo=64, hi=400)
    b = iga.Batch()
    b.submit(jobs)
    best, ms = b.autotune(reps=2)
    assert best in (4, 8, 16) and ms > 0
    b.flush()
    b.wait()
    for p, ne, u, m, l in jobs:
        rm, rl = _reference(iga, p, ne, u, best)
        torch.cuda.synchronize()
        assert torch.equal(m, rm) and torch.equal(l, rl)
    b.close()


def test_capacity_budget_and_states(iga):
    import torch
    jobs = _jobs(5, seed=4, lo=10, hi=40)
    # capacity
    b = iga.Batch(max_jobs=3)
    assert b.try_submit(jobs) is None              # all or nothing
    t = b.submit(jobs[:3])
    assert b.try_submit(jobs[3:4]) is None         # queue full
    b.flush()                                      # the queued jobs move to the GPU
    t2 = b.submit(jobs[3:5])                        # and free the queue
    assert b.poll(t2[0]) == iga.JOB_QUEUED
    b.flush()                                       # waits for the first launch first
    assert all(b.poll(x) == iga.JOB_DONE for x in t)
    b.wait()
    assert all(b.poll(x) == iga.JOB_DONE for x in t + t2)
    with pytest.raises(iga.IGAError):
        b.poll(10_000)
    b.close()
    # memory budget: u + mass + lap of the first job only
    first = jobs[0][2].numel() * 8 * 3
    b = iga.Batch(mem_budget_bytes=first)
    t = b.submit(jobs[:1])
    assert b.try_submit(jobs[1:2]) is None
    b.flush()
    assert b.try_submit(jobs[1:2]) is None         # the running job still holds its bytes
    b.wait()
    assert b.try_submit(jobs[1:2]) is not None
    b.flush()
    b.wait()
    b.close()


def test_invalid_jobs_rejected(iga):
    import torch
    u = torch.zeros(6, 6, dtype=torch.float64, device="cuda")
    m, l = torch.empty_like(u), torch.empty_like(u)
    b = iga.Batch()
    for bad, code in (((4, (2, 2), u, m, l), iga.IGA_E_UNSUPPORTED), ((2, (0, 4), u, m, l), iga.IGA_E_INVAL),
                      ((2, (4, 4), u, m, m), iga.IGA_E_INVAL)):
        with pytest.raises(iga.IGAError) as e:
            b.submit([bad])
        assert e.value.code == code
    b.close()
