"""Pins of the oracle's right-hand-side generation and explicit step (CPU only).

 * P14: the 2D/3D generation (direct sum over the (p+1)^d local products at every
   Gauss point) equals the Kronecker combination of the 1D matrices (Section 3:
   the 2D/3D rows are tensor products; Section 4.1: the alternating-directions
   structure), on anisotropic meshes so that a transposed axis fails;
 * P12: brute force -- 1D rows with polynomial data equal exact-rational integrals;
 * P9: int_S Lap u_h = u_h'(end of S) - u_h'(start of S) (fundamental theorem of
   calculus; no quadrature of B'' involved);
 * closed forms for the source term: int_S 1 = |S|, int B_i = (t_{i+p+1}-t_i)/(p+1),
   separable monomials, and the sine source within the Gauss error bound;
 * P13: explicit step (Section 4.2): constants are preserved, dt = 0 gives the
   lumped projection, and a resumed run equals the uninterrupted one bitwise.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from exact_bspline import ExactSpace


def _kron_apply(mats, u):
    """sum over the tensor product of per-axis matrices (x, y, z order) applied to u."""
    if len(mats) == 1:
        return mats[0] @ u
    if len(mats) == 2:
        return mats[1] @ u @ mats[0].T
    return np.einsum("zk,yj,xi,kji->zyx", mats[2], mats[1], mats[0], u)


def _mats(orc, pb, form):
    out = []
    for a in range(pb.dim):
        kw = dict(lo=pb.lo[a], hi=pb.hi[a])
        if form == orc.PG:
            M = orc.matrix_1d(pb.p, pb.ne[a], pb.nq[a], orc.MAT_PG_MASS, span=pb._spans[a], **kw)
            D = orc.matrix_1d(pb.p, pb.ne[a], pb.nq[a], orc.MAT_PG_LAP, span=pb._spans[a], **kw)
        else:
            M = orc.matrix_1d(pb.p, pb.ne[a], pb.nq[a], orc.MAT_GAL_MASS, **kw)
            kind = orc.MAT_GAL_LAP if form == orc.GALERKIN_LAPLACIAN else orc.MAT_GAL_BYPARTS
            D = orc.matrix_1d(pb.p, pb.ne[a], pb.nq[a], kind, **kw)
        out.append((M, D))
    return out


CASES = [
    (1, 2, (9,)), (1, 3, (7,)),
    (2, 2, (5, 3)), (2, 3, (4, 6)),
    (3, 2, (3, 4, 2)), (3, 3, (2, 3, 4)),
]


@pytest.mark.parametrize("dim,p,ne", CASES)
@pytest.mark.parametrize("form", [0, 1, 2])
def test_tensor_rows_equal_kronecker(orc, dim, p, ne, form):
    """P14."""
    pb = orc.Problem(dim=dim, p=p, ne=ne, nq=[p + 1, p + 2, p + 1][:dim],
                     lo=(0.0, -1.0, 0.5), hi=(1.0, 0.5, 2.5),
                     span_kind="support" if dim != 2 else "element")
    rng = np.random.default_rng(11)
    u = rng.standard_normal(pb.coef_shape())
    alpha, beta = 0.7, -1.3
    got = orc.rhs(pb, form, u, alpha, beta)
    mats = _mats(orc, pb, form)
    ref = alpha * _kron_apply([m for m, _ in mats], u)
    for t in range(dim):
        ref = ref + beta * _kron_apply([d if a == t else m for a, (m, d) in enumerate(mats)], u)
    np.testing.assert_allclose(got, ref, atol=1e-11 * np.abs(ref).max())
    # slabs of the outer axis reproduce the full result
    r0, r1 = 1, got.shape[0] - 1
    np.testing.assert_array_equal(orc.rhs(pb, form, u, alpha, beta, rows=(r0, r1)), got[r0:r1])


@pytest.mark.parametrize("p,ne", [(2, 4), (2, 7), (3, 5)])
def test_1d_rows_equal_exact_integrals(orc, p, ne):
    """P12: random coefficients, cubic f; Gauss exact for nq = p + 2."""
    sp = ExactSpace(p, ne)
    rng = np.random.default_rng(3)
    u = rng.integers(-5, 6, size=ne + p).astype(float)
    fpoly = (Fr(1, 3), Fr(-2), Fr(1, 2), Fr(5, 4))   # 1/3 - 2x + x^2/2 + 5x^3/4
    nq = p + 2
    xi = np.polynomial.legendre.leggauss(nq)[0]
    xs = ((np.arange(ne)[:, None] + (xi[None, :] + 1) / 2) / ne).ravel()
    table = sum(float(c) * xs ** k for k, c in enumerate(fpoly))
    pb = orc.Problem(dim=1, p=p, ne=(ne,), nq=(nq,))
    first, last = pb._spans[0]
    alpha, beta, gamma = 2.0, 0.5, -1.5
    # PG
    PM, PD = np.array(sp.pg("mass", first, last)), np.array(sp.pg("lap", first, last))
    ex = [alpha * sum(PM[r][j] * Fr(u[j]) for j in range(ne + p)) +
          beta * sum(PD[r][j] * Fr(u[j]) for j in range(ne + p)) +
          gamma * sp.span_integral(int(first[r]), int(last[r]), fpoly) for r in range(len(first))]
    got = orc.rhs(pb, orc.PG, u, alpha, beta, gamma, f_table=table)
    np.testing.assert_allclose(got, [float(v) for v in ex], atol=1e-12 * ne ** 2)
    # Galerkin, both forms
    for form, name in ((orc.GALERKIN_LAPLACIAN, "lap"), (orc.GALERKIN_BYPARTS, "byparts")):
        M, K = sp.gal("mass"), sp.gal(name)
        ex = [alpha * sum(M[i][j] * Fr(u[j]) for j in range(ne + p)) +
              beta * sum(K[i][j] * Fr(u[j]) for j in range(ne + p)) +
              gamma * sp.weighted(i, fpoly) for i in range(ne + p)]
        got = orc.rhs(pb, form, u, alpha, beta, gamma, f_table=table)
        np.testing.assert_allclose(got, [float(v) for v in ex], atol=1e-12 * ne ** 2)
    # the 20-point rule gives the same rows
    pb20 = orc.Problem(dim=1, p=p, ne=(ne,), nq=(20,))
    np.testing.assert_allclose(orc.rhs(pb20, orc.PG, u, alpha, beta),
                               orc.rhs(pb, orc.PG, u, alpha, beta), atol=1e-12 * ne ** 2)


@pytest.mark.parametrize("p,ne", [(2, 9), (3, 12)])
@pytest.mark.parametrize("nq", [2, 3, 4])
def test_pg_laplacian_flux_identity(orc, p, ne, nq):
    """P9: int_S Lap u_h = u_h'(x_{t+1}) - u_h'(x_s).  B'' is a polynomial of degree p-2 on
    every element, so any rule with 2 nq - 1 >= p - 2 integrates it exactly."""
    pb = orc.Problem(dim=1, p=p, ne=(ne,), nq=(nq,))
    u = np.random.default_rng(5).standard_normal(ne + p)
    got = orc.rhs(pb, orc.PG, u, beta=1.0)
    first, last = pb._spans[0]
    for r, (s, t) in enumerate(zip(first, last)):
        d1 = orc.basis_eval(p, ne, (t + 1) / ne, nder=1)[1] @ u
        d0 = orc.basis_eval(p, ne, s / ne, nder=1)[1] @ u
        assert abs(got[r] - (d1 - d0)) <= 1e-12 * ne * np.abs(u).sum()


@pytest.mark.parametrize("dim,p,ne", CASES)
def test_source_closed_forms(orc, dim, p, ne):
    """f = 1: PG rows are |S_r|; Galerkin rows are prod_a (t_{i+p+1}-t_i)/(p+1)."""
    nq = [p + 1] * dim
    pb = orc.Problem(dim=dim, p=p, ne=ne, nq=nq)
    ones = np.ones(pb.gauss_shape())
    got = orc.rhs(pb, orc.PG, None, gamma=2.0, f_table=ones)
    lens = orc.span_lengths(pb)
    ref = 2.0 * _kron_apply([np.diag(l) for l in lens], np.ones(pb.shape(orc.PG)))
    np.testing.assert_allclose(got, ref, rtol=1e-14)
    ints = []
    for a in range(dim):
        n = ne[a]
        t = np.concatenate([np.zeros(p), np.arange(n + 1) / n, np.ones(p)])
        ints.append(np.diag((t[p + 1:] - t[:n + p]) / (p + 1)))
    for form in (orc.GALERKIN_BYPARTS, orc.GALERKIN_LAPLACIAN):
        got = orc.rhs(pb, form, None, gamma=1.0, f_table=ones)
        np.testing.assert_allclose(got, _kron_apply(ints, np.ones(got.shape)), rtol=1e-14)


def test_source_table_layout_separable_monomial(orc):
    """A Gauss table holding x^2 y^3 z gives exact separable span integrals (x fastest)."""
    p, ne, nq = 2, (5, 4, 3), (3, 3, 3)
    pb = orc.Problem(dim=3, p=p, ne=ne, nq=nq)
    pts = []
    for a in range(3):
        xi = np.polynomial.legendre.leggauss(nq[a])[0]
        pts.append(((np.arange(ne[a])[:, None] + (xi[None, :] + 1) / 2) / ne[a]).ravel())
    table = (pts[2][:, None, None] * pts[1][None, :, None] ** 3 * pts[0][None, None, :] ** 2)
    got = orc.rhs(pb, orc.PG, None, gamma=1.0, f_table=table)
    first = [pb._spans[a][0] for a in range(3)]
    last = [pb._spans[a][1] for a in range(3)]
    powers = (2, 3, 1)
    ints = []
    for a in range(3):
        k = powers[a]
        x0 = first[a] / ne[a]
        x1 = (last[a] + 1) / ne[a]
        ints.append((x1 ** (k + 1) - x0 ** (k + 1)) / (k + 1))
    ref = ints[2][:, None, None] * ints[1][None, :, None] * ints[0][None, None, :]
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("dim,p,ne", [(1, 2, (16,)), (2, 3, (6, 9)), (3, 2, (4, 3, 5))])
def test_sine_source_within_gauss_error_bound(orc, dim, p, ne):
    """amp prod sin(pi x_a): PG rows against the exact separable integral, within the
    n-point Gauss error bound (b-a)^{2n+1} (n!)^4 / ((2n+1) ((2n)!)^3) max|f^{(2n)}| per
    element and axis; and the d-D rows equal the product of the 1D rows."""
    nq = 3
    pb = orc.Problem(dim=dim, p=p, ne=ne, nq=[nq] * dim)
    amp = 1.7
    got = orc.rhs(pb, orc.PG, None, gamma=1.0, sin_amp=amp)
    ints1, rows1 = [], []
    for a in range(dim):
        f, l = pb._spans[a]
        x0, x1 = f / ne[a], (l + 1) / ne[a]
        ints1.append((np.cos(np.pi * x0) - np.cos(np.pi * x1)) / np.pi)
        p1 = orc.Problem(dim=1, p=p, ne=(ne[a],), nq=(nq,))
        rows1.append(orc.rhs(p1, orc.PG, None, gamma=1.0, sin_amp=1.0))
    ref = amp * _kron_apply([np.diag(v) for v in ints1], np.ones(got.shape))
    sep = amp * _kron_apply([np.diag(v) for v in rows1], np.ones(got.shape))
    np.testing.assert_allclose(got, sep, rtol=1e-13, atol=1e-15)
    hmax = max(1.0 / n for n in ne)
    n = nq
    per_elem = hmax ** (2 * n + 1) * math.factorial(n) ** 4 / (
        (2 * n + 1) * math.factorial(2 * n) ** 3) * np.pi ** (2 * n)
    bound = amp * dim * (p + 1) * per_elem * 1.0001
    assert np.abs(got - ref).max() <= bound
    assert np.abs(got - ref).max() > 0


@pytest.mark.parametrize("dim,p,ne", [(1, 3, (10,)), (2, 2, (6, 5)), (3, 3, (3, 4, 3))])
def test_explicit_step_invariants(orc, dim, p, ne):
    """P13 (Section 4.2 with the lumped left-hand side)."""
    pb = orc.Problem(dim=dim, p=p, ne=ne, nq=[p + 1] * dim)
    shape = pb.coef_shape()
    # constants are preserved exactly up to round-off (f = 0)
    u = np.full(shape, 3.25)
    out = orc.explicit_step(pb, u, dt=1e-3, nsteps=5)
    np.testing.assert_allclose(out, 3.25, rtol=1e-14)
    # dt = 0: one step is the lumped projection P_M u / |S|
    u = np.random.default_rng(2).standard_normal(shape)
    out = orc.explicit_step(pb, u, dt=0.0)
    lens = orc.span_lengths(pb)
    mats = [orc.matrix_1d(p, ne[a], p + 1, orc.MAT_PG_MASS) / lens[a][:, None] for a in range(dim)]
    np.testing.assert_allclose(out, _kron_apply(mats, u), atol=1e-13)
    # resume: 3 + 4 steps == 7 steps, bitwise
    f = np.random.default_rng(9).uniform(-1, 1, pb.gauss_shape())
    a = orc.explicit_step(pb, u, dt=1e-4, f_table=f, sin_amp=0.5, nsteps=7)
    b = orc.explicit_step(pb, u, dt=1e-4, f_table=f, sin_amp=0.5, nsteps=3)
    b = orc.explicit_step(pb, b, dt=1e-4, f_table=f, sin_amp=0.5, nsteps=4)
    np.testing.assert_array_equal(a, b)
    # one step equals the PG rows divided by |S|
    b1 = orc.rhs(pb, orc.PG, u, 1.0, 1e-4, 1e-4, f_table=f, sin_amp=0.5)
    inv = _kron_apply([np.diag(1.0 / l) for l in lens], b1)
    np.testing.assert_allclose(orc.explicit_step(pb, u, 1e-4, f_table=f, sin_amp=0.5), inv,
                               rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("p,ne", [(2, (7, 5)), (3, (6, 9)), (3, (1, 4))])
def test_quadratic_precision_closed_forms(orc, p, ne):
    """Quadratic precision of B-splines (coefficients = blossom of x^2 at the inner
    knots of each B-spline) makes u_h = x^2 + 3 y^2 exactly, so:
      PG rows (support spans):  int_S u_h = closed form, int_S Lap u_h = 8 |S|;
      Galerkin rows:            int B_i B_j Lap u_h = 8 int B_i int B_j (Laplacian form)
                                and the by-parts form differs from it only on the
                                boundary rows;
      explicit step (f = 0):    mean_S(u_h) + 8 dt."""
    from closed_forms import bspline_integrals, quad_coefs, support_span_moments
    nx, ny = ne
    u = quad_coefs(p, nx)[None, :] + 3.0 * quad_coefs(p, ny)[:, None]
    pb = orc.Problem(dim=2, p=p, ne=ne, nq=(p + 1, p + 1))
    wx, x2 = support_span_moments(p, nx, np.arange(nx + p))
    wy, y2 = support_span_moments(p, ny, np.arange(ny + p))
    area = wx[None, :] * wy[:, None]
    mass = x2[None, :] * wy[:, None] + 3.0 * wx[None, :] * y2[:, None]
    np.testing.assert_allclose(orc.rhs(pb, orc.PG, u, alpha=1.0), mass, rtol=1e-14)
    np.testing.assert_allclose(orc.rhs(pb, orc.PG, u, beta=1.0), 8.0 * area, rtol=1e-13)
    gi = 8.0 * bspline_integrals(p, nx)[None, :] * bspline_integrals(p, ny)[:, None]
    np.testing.assert_allclose(orc.rhs(pb, orc.GALERKIN_LAPLACIAN, u, beta=1.0), gi, rtol=1e-13)
    bp = orc.rhs(pb, orc.GALERKIN_BYPARTS, u, beta=1.0)
    inner = (slice(1, -1), slice(1, -1))
    if ny + p > 2 and nx + p > 2:
        np.testing.assert_allclose(bp[inner], gi[inner], rtol=1e-13)
    dt = 1e-3
    step = orc.explicit_step(pb, u, dt)
    np.testing.assert_allclose(step, mass / area + 8.0 * dt, rtol=1e-14)
