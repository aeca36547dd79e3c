"""GPU parity of the alternating-directions solve with the Galerkin mass (iga_solve) and
of the consistent-mass Galerkin Euler step (iga_galerkin_step) against the CPU oracle,
through the C ABI.

Tolerance: normwise relative error ||x_gpu - x_oracle||_inf / ||x_oracle||_inf <= 1e-12,
the bar of every other parity test.  A solve amplifies rounding by the condition number
of the Kronecker mass, kappa_inf = prod_a kappa_inf(M_a) (12.8 per axis for p = 2 and
33.6 for p = 3, flat in the element count), so the worst-case forward error bound d kappa
u (u = 2^-53) is 2.3e-13 for 2D p = 3 and 1.3e-11 for 3D p = 3; the measured differences
are of order 1e-15, far inside the bar.  The two reduced systems of the partitioned
solve differ by rounding only (the dropped coupling is below 2^-64): 1e-13."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from closed_forms import quad_coefs  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def iga(torch):
    from paper_1910_08535_amd import iga as m
    return m


def _rel(a, b):
    """Normwise relative error in the infinity norm."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _mesh(iga, dim, p, ne, lo=None, hi=None):
    lo = lo or [0.0] * dim
    hi = hi or [1.0] * dim
    return iga.Mesh(dim, p, ne, [p + 1] * dim, lo=lo, hi=hi)


SOLVE_CASES = [
    (1, 2, (37,), None, None),
    (1, 3, (2000,), (-1.0,), (3.0,)),              # long axis: repeated factor rows
    (2, 2, (5, 3), None, None),                    # no interior rows
    (2, 2, (45, 38), (0.0, -1.0), (2.0, 0.5)),
    (2, 3, (300, 40), None, None),                 # repeated rows along x
    (3, 2, (20, 17, 23), (0.0, 0.0, -2.0), (1.0, 0.5, 1.0)),
    (3, 3, (14, 19, 12), None, None),
    (3, 3, (130, 9, 7), None, None),               # repeated rows along x, 3D
    (3, 2, (6, 150, 11), None, None),              # repeated rows along y
    (3, 2, (8, 300, 9), None, None),               # y-lines in chunks of the segment kernel
    (1, 2, (1,), None, None),                      # one element: N = p + 1
    (2, 3, (1, 5), None, None),
    (3, 2, (1, 1, 1), (0.0, 1.0, 2.0), (0.5, 3.0, 2.25)),
    (2, 2, (800, 3), None, None),                  # x-lines longer than the on-chip limit
    (3, 3, (1000, 20, 12), None, None),            # long x-lines beside short y and z lines
    (3, 2, (1600, 90, 92), None, None),            # many x-lines too long for the segment kernel
    (2, 2, (1024, 1024), None, None),              # lines of two halves in both families
    (2, 3, (1300, 50), (0.0, 0.0), (2.0, 1.0)),
    (1, 2, (5000,), (0.0,), (2.0,)),               # one line: interior chunks of equal length
    (1, 3, (4000,), None, None),                   # one interior chunk between the end chunks
    (1, 3, (300,), None, None),                    # one line of 303 rows: short chunks
    (2, 3, (4, 300), None, None),                  # y-lines partitioned, x-lines not
    (2, 3, (70, 500), (0.0, -1.0), (1.0, 1.0)),    # y-lines in chunks of the segment kernel
]


@pytest.mark.parametrize("dim,p,ne,lo,hi", SOLVE_CASES)
def test_solve_parity(orc, torch, iga, dim, p, ne, lo, hi):
    print(f"solve dim={dim} p={p} ne={ne}", flush=True)
    mesh = _mesh(iga, dim, p, ne, lo, hi)
    pb = orc.Problem(dim, p, ne, [p + 1] * dim, lo or [0.0] * dim, hi or [1.0] * dim)
    b = np.random.default_rng(21).standard_normal(pb.coef_shape())
    bd = torch.from_numpy(b).cuda()
    x = mesh.solve(bd).cpu().numpy()
    ref = orc.ads_solve(pb, b)
    assert _rel(x, ref) < TOL
    # in place gives the same bits, and b is left alone out of place
    assert np.array_equal(bd.cpu().numpy(), b)
    y = bd.clone()
    mesh.solve(y, out=y)
    assert torch.equal(y.cpu(), torch.from_numpy(x))
    # both Galerkin forms share the mass
    z = mesh.solve(bd, form=iga.GALERKIN_BYPARTS)
    assert torch.equal(z.cpu(), torch.from_numpy(x))
    mesh.close()


# partitioned families, with the scheme each axis takes by default (L: whole lines,
# E: partitioned with the exact reduced sweeps, B: partitioned with the block-diagonal
# reduced system): 2D lines in balanced chunks of the segment kernel (p = 3 at least 76
# rows each, so that the dropped spike ends stay below 2^-64), single lines in short
# interior chunks, families of 2 to 63 lines with one thread per chunk (p = 3: chunks of
# 65 rows keep dropped entries above the bound, exact sweeps; chunks of 75-76 rows do not)
L, E, B = 1, 2, 3
PART_CASES = [
    (2, 2, (1024, 1024), None, None, (B, B)),
    (2, 3, (1300, 50), (0.0, 0.0), (2.0, 1.0), (E, L)),
    (1, 2, (5000,), (0.0,), (2.0,), (B,)),
    (1, 3, (4000,), None, None, (B,)),
    (1, 3, (300,), None, None, (B,)),
    (2, 3, (4, 300), None, None, (L, B)),
    (2, 3, (70, 500), (0.0, -1.0), (1.0, 1.0), (L, B)),
    (2, 2, (300, 200), None, None, (B, B)),
    (2, 3, (200, 200), None, None, (B, B)),   # the p = 3 cap binds: 2 chunks, not 3
    (1, 2, (4118,), None, None, (B,)),   # a workgroup boundary inside the last chunk: two solve it
    (1, 3, (4147,), None, None, (B,)),   # the same with a last chunk of 70 rows (two waves)
    (1, 2, (4178,), None, None, (B,)),   # a workgroup boundary inside the chunk before the last
]


@pytest.mark.parametrize("dim,p,ne,lo,hi,schemes", PART_CASES)
def test_solve_exact_reduced_system(orc, torch, iga, dim, p, ne, lo, hi, schemes):
    """The partitioned solve with its reduced system taken whole (the context setting
    TILE_SOLVE_EXACT = 1: block sweeps along each line) and by default (block diagonal
    where every dropped spike entry is below 2^-64): both agree with the oracle and with
    each other to rounding, and each axis reports the scheme it took.  The setting is
    refused once a solve has run."""
    print(f"solve exact reduced dim={dim} p={p} ne={ne}", flush=True)
    pb = orc.Problem(dim, p, ne, [p + 1] * dim, lo or [0.0] * dim, hi or [1.0] * dim)
    b = np.random.default_rng(23).standard_normal(pb.coef_shape())
    bd = torch.from_numpy(b).cuda()
    ref = orc.ads_solve(pb, b)
    mesh = _mesh(iga, dim, p, ne, lo, hi)
    assert [mesh.solve_info(a)[0] for a in range(dim)] == [iga.SOLVE_NONE] * dim
    x = mesh.solve(bd).cpu().numpy()
    got = tuple(mesh.solve_info(a)[0] for a in range(dim))
    mesh.close()
    assert got == schemes, (got, schemes)
    mesh = _mesh(iga, dim, p, ne, lo, hi)
    assert mesh.get_tile(iga.TILE_SOLVE_EXACT) == 0
    mesh.set_tile(iga.TILE_SOLVE_EXACT, 1)
    xe = mesh.solve(bd).cpu().numpy()
    got_e = tuple(mesh.solve_info(a)[0] for a in range(dim))
    assert mesh.get_tile(iga.TILE_SOLVE_EXACT) == 1
    with pytest.raises(iga.IGAError):
        mesh.set_tile(iga.TILE_SOLVE_EXACT, 0)
    mesh.close()
    assert got_e == tuple(E if s == B else s for s in schemes), got_e
    print(f"  errors: default {_rel(x, ref):.2e} exact {_rel(xe, ref):.2e} "
          f"between {_rel(x, xe):.2e}", flush=True)
    assert _rel(x, ref) < TOL
    assert _rel(xe, ref) < TOL
    assert _rel(x, xe) < 1e-13


def test_first_solve_not_captured(torch, iga):
    """The first solve builds tables, so it is refused during stream capture; after an
    uncaptured solve, a captured one replays the eager result, bit for bit."""
    st = torch.cuda.Stream()
    mesh = iga.Mesh(2, 2, (300, 200), [3, 3], stream=st)
    gen = torch.Generator(device="cuda").manual_seed(26)
    b = torch.randn(mesh.coef_shape(), dtype=torch.float64, device="cuda", generator=gen)
    x = torch.empty_like(b)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(iga.IGAError) as e:
        with torch.cuda.graph(g, stream=st):
            mesh.solve(b, out=x)
    assert e.value.code == iga.IGA_E_INVAL
    assert mesh.solve_info(0)[0] == iga.SOLVE_NONE
    with torch.cuda.stream(st):
        ref = mesh.solve(b).clone()
    st.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        mesh.solve(b, out=x)
    for k in range(3):
        x.zero_()
        b.add_(0.0)   # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, ref), k
    mesh.close()


def test_solve_error_codes(torch, iga):
    mesh = _mesh(iga, 2, 2, (8, 8))
    b = torch.zeros(mesh.coef_shape(), dtype=torch.float64, device="cuda")
    with pytest.raises(iga.IGAError) as e:
        mesh.solve(b, form=iga.PG)
    assert e.value.code == iga.IGA_E_SINGULAR
    with pytest.raises(iga.IGAError) as e:
        mesh.galerkin_step(b, 1e-4, form=iga.PG)
    assert e.value.code == iga.IGA_E_SINGULAR
    L = iga.lib()
    assert L.iga_solve(mesh.h, 7, b.data_ptr(), b.data_ptr()) == iga.IGA_E_INVAL
    assert L.iga_solve(mesh.h, 1, None, b.data_ptr()) == iga.IGA_E_INVAL
    assert L.iga_galerkin_step(mesh.h, 1, b.data_ptr(), 1e-4, None, -1) == iga.IGA_E_INVAL
    mesh.close()


def _gauss_table(orc, pb, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=pb.gauss_shape())


@pytest.mark.parametrize("dim,p,ne,form", [
    (1, 3, (60,), 1),
    (1, 2, (4000,), 0),            # one line in chunks: end chunks on side streams
    (2, 2, (40, 33), 1),
    (2, 3, (21, 34), 0),
    (3, 2, (12, 10, 9), 0),
    (3, 3, (11, 9, 13), 1),
])
def test_galerkin_step_parity(orc, torch, iga, dim, p, ne, form):
    print(f"galerkin step dim={dim} p={p} ne={ne} form={form}", flush=True)
    mesh = _mesh(iga, dim, p, ne)
    pb = orc.Problem(dim, p, ne, [p + 1] * dim)
    u0 = np.random.default_rng(22).standard_normal(pb.coef_shape())
    tab = _gauss_table(orc, pb, 23)
    h = 1.0 / max(ne)
    dt = 1e-3 * h * h
    ref = orc.galerkin_step(pb, u0, dt, form, f_table=tab, sin_amp=0.7, nsteps=3)
    u = torch.from_numpy(u0).cuda()
    mesh.galerkin_step(u, dt, form=form, f_table=torch.from_numpy(tab).cuda(), sin_amp=0.7,
                       nsteps=3)
    assert _rel(u.cpu().numpy(), ref) < TOL
    mesh.close()


@pytest.mark.parametrize("p", [2, 3])
def test_solve_full_size_3d(orc, torch, iga, p):
    """256^3 elements (the size of the paper's projection table), every value against
    the oracle; and the solve undoes the GPU mass application."""
    ne = (256, 256, 256)
    print(f"solve full size p={p} ne={ne}", flush=True)
    mesh = _mesh(iga, 3, p, ne)
    pb = orc.Problem(3, p, ne, [p + 1] * 3)
    b = np.random.default_rng(24).standard_normal(pb.coef_shape())
    x = mesh.solve(torch.from_numpy(b).cuda())
    ref = orc.ads_solve(pb, b)
    assert _rel(x.cpu().numpy(), ref) < TOL
    del ref
    u0 = torch.from_numpy(b).cuda()
    m, _ = mesh.apply(iga.GALERKIN_LAPLACIAN, u0, lap=False)
    back = mesh.solve(m, out=m)
    assert _rel(back.cpu().numpy(), b) < TOL
    mesh.close()


@pytest.mark.parametrize("dim,p,ne", [(2, 2, (1024, 1024)), (3, 3, (128, 128, 128))])
def test_galerkin_step_quadratic_full_size(torch, iga, dim, p, ne):
    """u = sum_a x_a^2: Lap u = 2 dim, so every Laplacian-form step adds 2 dim dt to each
    coefficient (closed form, at the benchmark sizes)."""
    print(f"galerkin step quadratic dim={dim} p={p} ne={ne}", flush=True)
    mesh = _mesh(iga, dim, p, ne)
    u0 = np.zeros(mesh.coef_shape())
    for a in range(dim):
        shape = [1] * dim
        shape[dim - 1 - a] = ne[a] + p
        u0 = u0 + quad_coefs(p, ne[a]).reshape(shape)
    dt = 1e-6
    u = torch.from_numpy(u0).cuda()
    mesh.galerkin_step(u, dt, form=iga.GALERKIN_LAPLACIAN, nsteps=2)
    d = u.cpu().numpy() - u0
    assert np.max(np.abs(d - 2 * 2 * dim * dt)) < 1e-11
    mesh.close()


@pytest.mark.parametrize("p", [2, 3])
def test_solve_1d_long_undoes_mass(torch, iga, p):
    """10^6 elements in 1D (one line of 10^6 + p rows, solved in chunks): the solve of the
    GPU mass rows of u gives u back."""
    ne = (1000000,)
    print(f"solve 1D long p={p}", flush=True)
    mesh = _mesh(iga, 1, p, ne)
    u = torch.randn(mesh.coef_shape(), dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(25))
    m, _ = mesh.apply(iga.GALERKIN_LAPLACIAN, u, lap=False)
    back = mesh.solve(m)
    err = ((back - u).abs().max() / u.abs().max()).item()
    assert err < TOL, err
    mesh.close()
