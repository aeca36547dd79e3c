"""GPU parity of the refined-test-space Petrov-Galerkin rows (IGA_SPANS_REFINED) and of
their solve (iga_solve with IGA_PG, banded LU of the square PG mass) against the CPU
oracle, through the C ABI.

Tolerances: normwise relative error in the infinity norm, rows 1e-12, as for every other
form.  A solve amplifies rounding by kappa_inf = prod_a kappa_inf(P_a) of the refined PG
mass factors (the infinity-norm condition numbers, computed from the oracle's own
matrices in the test), so the bar of a solve is max(1e-12, 8 d kappa_inf u)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


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


def _mesh(iga, dim, p, ne, rho, lo=None, hi=None):
    return iga.Mesh(dim, p, ne, [p + 1] * dim, lo=lo, hi=hi, spans="refined", refine=rho)


def _band(M, p):
    N = M.shape[0]
    out = np.zeros((N, 2 * p + 1))
    for r in range(N):
        for k in range(2 * p + 1):
            c = r + k - p
            if 0 <= c < M.shape[1]:
                out[r, k] = M[r, c]
    return out


@pytest.mark.parametrize("p,ne,rho", [(2, (13, 7, 9), (4, 8, 5)), (3, (11, 6, 8), (4, 6, 7))])
def test_refined_bands(orc, torch, iga, p, ne, rho):
    lo, hi = [0.0, -1.0, 2.0], [1.0, 2.0, 2.5]
    mesh = _mesh(iga, 3, p, ne, rho, lo, hi)
    bands = mesh.assemble(iga.PG, iga.OP_LAPLACE).cpu().numpy()
    for a in range(3):
        N = ne[a] + p
        for f, kind in ((0, orc.MAT_PG_MASS), (1, orc.MAT_PG_LAP)):
            want = _band(orc.refined_matrix_1d(p, ne[a], rho[a], p + 1, kind, lo[a], hi[a]), p)
            got = bands[a, f, :N]
            assert _rel(got, want) < 1e-12, (a, f)
    mesh.close()


@pytest.mark.parametrize("dim,p,ne,rho", [
    (1, 3, (40,), (4,)),
    (2, 2, (37, 29), (4, 5)),
    (2, 3, (21, 33), (8, 4)),
    (3, 2, (9, 12, 7), (4, 4, 6)),
    (3, 3, (8, 7, 10), (4, 5, 4)),
    (1, 2, (1,), (4,)),                           # one trial element
    (2, 3, (1, 3), (4, 64)),                      # the largest refinement
])
def test_refined_rows(orc, torch, iga, dim, p, ne, rho):
    print(f"refined rows dim={dim} p={p} ne={ne} rho={rho}", flush=True)
    mesh = _mesh(iga, dim, p, ne, rho)
    pb = orc.Problem(dim, p, ne, [p + 1] * dim)
    u = np.random.default_rng(61).standard_normal(pb.coef_shape())
    want = orc.refined_rhs(pb, rho, u, alpha=0.8, beta=-0.3, gamma=1.7, sin_amp=0.9)
    got = mesh.rhs(iga.PG, torch.from_numpy(u).cuda(), 0.8, -0.3, 1.7, sin_amp=0.9).cpu().numpy()
    assert _rel(got, want) < 1e-12
    m, l = mesh.apply(iga.PG, torch.from_numpy(u).cuda())
    assert _rel(m.cpu().numpy(), orc.refined_rhs(pb, rho, u, alpha=1.0)) < 1e-12
    assert _rel(l.cpu().numpy(), orc.refined_rhs(pb, rho, u, beta=1.0)) < 1e-12
    mesh.close()


def _kappa(orc, pb, rho):
    k = 1.0
    for a in range(pb.dim):
        k *= np.linalg.cond(orc.refined_matrix_1d(pb.p, pb.ne[a], rho[a], pb.nq[a], orc.MAT_PG_MASS,
                                                  pb.lo[a], pb.hi[a]), np.inf)
    return k


@pytest.mark.parametrize("dim,p,ne,rho", [
    (1, 2, (50,), (4,)),
    (2, 3, (30, 17), (4, 8)),
    (3, 2, (12, 9, 14), (4, 6, 4)),
    (3, 3, (10, 8, 9), (4, 4, 5)),
    (2, 2, (1, 2), (3, 4)),                       # the smallest sizes and refinements
])
def test_refined_solve(orc, torch, iga, dim, p, ne, rho):
    print(f"refined solve dim={dim} p={p} ne={ne} rho={rho}", flush=True)
    mesh = _mesh(iga, dim, p, ne, rho)
    pb = orc.Problem(dim, p, ne, [p + 1] * dim)
    b = np.random.default_rng(62).standard_normal(pb.coef_shape())
    want = orc.refined_solve(pb, rho, b)
    got = mesh.solve(torch.from_numpy(b).cuda(), form=iga.PG).cpu().numpy()
    tol = max(1e-12, 8 * dim * _kappa(orc, pb, rho) * U)
    assert _rel(got, want) < tol
    # the consistent refined-PG Euler step: rows of u + dt Lap u + dt f, then the solve
    u = np.random.default_rng(63).standard_normal(pb.coef_shape())
    dt = 1e-4 / max(ne) ** 2
    ref = orc.refined_solve(pb, rho, orc.refined_rhs(pb, rho, u, 1.0, dt, dt, sin_amp=0.5))
    ud = torch.from_numpy(u).cuda()
    mesh.galerkin_step(ud, dt, form=iga.PG, sin_amp=0.5)
    assert _rel(ud.cpu().numpy(), ref) < tol
    mesh.close()


@pytest.mark.parametrize("dim,p,ne,rho", [(2, 2, (1024, 1024), (4, 4)), (3, 3, (128, 128, 128), (4, 4, 4))])
def test_refined_solve_undoes_mass_full_size(orc, torch, iga, dim, p, ne, rho):
    """At the benchmark sizes: the PG mass rows of u, solved with the refined PG solve,
    give u back (bar: max(1e-11, 8 d kappa_inf u))."""
    print(f"refined full size dim={dim} p={p}", flush=True)
    mesh = _mesh(iga, dim, p, ne, rho)
    u = torch.randn(mesh.coef_shape(), dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(64))
    m, _ = mesh.apply(iga.PG, u, lap=False)
    back = mesh.solve(m, form=iga.PG, out=m)
    err = ((back - u).abs().max() / u.abs().max()).item()
    tol = max(1e-11, 8 * dim * _kappa(orc, orc.Problem(dim, p, ne, [p + 1] * dim), rho) * U)
    print(f"  error {err:.2e} bar {tol:.2e}", flush=True)
    assert err < tol, (err, tol)
    mesh.close()


def test_refined_error_codes(torch, iga):
    mesh = _mesh(iga, 2, 2, (8, 8), (4, 4))
    L = iga.lib()
    b = torch.zeros(mesh.coef_shape(), dtype=torch.float64, device="cuda")
    tab = torch.zeros((24, 24), dtype=torch.float64, device="cuda")
    src = iga.Source()
    src.table = tab.data_ptr()
    src.sin_amp = 0.0
    import ctypes as C
    assert L.iga_rhs(mesh.h, iga.PG, None, 0.0, 0.0, 1.0, C.byref(src), b.data_ptr()) == iga.IGA_E_UNSUPPORTED
    side = (iga.Side * 1)(iga.Side(0, None, 1.0))
    assert L.iga_boundary_terms(mesh.h, iga.PG, 1, side, None, 0.0, 1.0, b.data_ptr()) == iga.IGA_E_UNSUPPORTED
    # Galerkin forms on a refined context are the ordinary ones
    assert L.iga_rhs(mesh.h, iga.GALERKIN_BYPARTS, None, 0.0, 0.0, 1.0, C.byref(src), b.data_ptr()) == 0
    mesh.close()
    plain = iga.Mesh(2, 2, (8, 8), (3, 3))
    with pytest.raises(iga.IGAError) as e:
        plain.solve(b, form=iga.PG)
    assert e.value.code == iga.IGA_E_SINGULAR
    plain.close()
