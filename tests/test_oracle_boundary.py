"""Pins of the oracle's boundary terms for Neumann conditions and of its Dirichlet row
replacement (the mixed Laplace problem of Section 4.3), against facts of the
mathematics: the divergence theorem linking the Laplacian and by-parts Galerkin forms,
closed-form normal fluxes of polynomials the splines reproduce, closed-form integrals
of a linear G over spans (which also fixes the layout of a side's table), and the
discrete mixed system satisfied by an exact spline solution."""
import numpy as np
import pytest

from closed_forms import bspline_integrals, lin_coefs, quad_coefs

ALL = lambda dim: [dict(axis=a, hi=h) for a in range(dim) for h in (False, True)]  # noqa: E731


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("dim,p,ne,lo,hi", [
    (1, 2, (7,), (0.0,), (2.0,)),
    (2, 2, (5, 4), (0.0, -1.0), (1.0, 1.5)),
    (2, 3, (6, 5), (0.0, 0.0), (1.0, 1.0)),
    (3, 3, (4, 3, 5), (0.0, 0.0, 0.0), (1.0, 2.0, 0.5)),
])
def test_galerkin_divergence_identity(orc, dim, p, ne, lo, hi):
    """int B_i Lap u - int_{boundary} B_i du/dn = -int grad B_i . grad u: the Laplacian
    form minus the flux over every side is the by-parts form."""
    pb = orc.Problem(dim, p, ne, [p + 1] * dim, lo, hi)
    u = np.random.default_rng(31).standard_normal(pb.coef_shape())
    lap = orc.rhs(pb, orc.GALERKIN_LAPLACIAN, u, 0.0, 1.0, 0.0)
    bp = orc.rhs(pb, orc.GALERKIN_BYPARTS, u, 0.0, 1.0, 0.0)
    flux = orc.boundary_terms(pb, orc.GALERKIN_LAPLACIAN, ALL(dim), u, alpha=1.0)
    assert _rel(lap - flux, bp) < 1e-12


def _spans_len(orc, pb, b):
    f, l = pb._spans[b]
    return (l - f + 1) / pb.ne[b]


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("form", [0, 2])
def test_closed_form_fluxes_2d(orc, p, form):
    """u = x^2 + (1-x)^2 + 3 y^2 on the unit square: du/dn = 2 on x = 1 and on x = 0
    (outward normal -x), 6 on y = 1 and 0 on y = 0.  A side's rows are then that
    constant times the test function's integral along the side: |S_r| of the tangential
    span (PG, rows whose span reaches the side) or int B_r (Galerkin, the end row)."""
    ne = (6, 5)
    pb = orc.Problem(2, p, ne, (p + 1, p + 1))
    one = np.ones(ne[0] + p)
    cx = quad_coefs(p, ne[0]) + (one - 2 * lin_coefs(p, ne[0]) + quad_coefs(p, ne[0]))
    u = cx[None, :] + 3.0 * quad_coefs(p, ne[1])[:, None]
    flux = {(a, h): 2.0 if a == 0 else (6.0 if h else 0.0) for a in (0, 1) for h in (False, True)}
    for (a, h), dn in flux.items():
        got = orc.boundary_terms(pb, form, [dict(axis=a, hi=h)], u, alpha=1.0)
        b = 1 - a
        tang = _spans_len(orc, pb, b) if form == orc.PG else bspline_integrals(p, ne[b])
        if form == orc.PG:
            f, l = pb._spans[a]
            norm = ((l == ne[a] - 1) if h else (f == 0)).astype(float)
        else:
            norm = np.zeros(ne[a] + p)
            norm[-1 if h else 0] = 1.0
        want = dn * np.multiply.outer(norm, tang)          # (rows_a, rows_b)
        want = want.T if a == 0 else want                  # numpy order (rows_y, rows_x)
        assert np.allclose(got, want, rtol=1e-12, atol=1e-13), (a, h)


def test_side_table_layout_2d_and_3d(orc):
    """A linear G on a side: int over the span of (x + 10 y) is closed-form; a swapped or
    mis-strided table gives other values.  PG support spans on the unit square/cube."""
    p = 2
    pb = orc.Problem(2, p, (6, 5), (3, 3))
    xi, _ = np.polynomial.legendre.leggauss(3)
    xq = ((np.arange(6)[:, None] + (xi[None, :] + 1) / 2) / 6).ravel()
    got = orc.boundary_terms(pb, orc.PG, [dict(axis=1, hi=True, g_table=xq)], beta=1.0)
    f, l = pb._spans[0]
    a, b = f / 6, (l + 1) / 6
    want_x = (b - a) * (a + b) / 2                        # int_{S_r} x dx
    fy, ly = pb._spans[1]
    touch = (ly == 4).astype(float)
    assert np.allclose(got, np.multiply.outer(touch, want_x), rtol=1e-12, atol=1e-14)

    pb3 = orc.Problem(3, p, (4, 3, 5), (3, 3, 3))
    gx = ((np.arange(4)[:, None] + (xi[None, :] + 1) / 2) / 4).ravel()
    gy = ((np.arange(3)[:, None] + (xi[None, :] + 1) / 2) / 3).ravel()
    tab = gx[None, :] + 10.0 * gy[:, None]                # face z = 1: x fastest
    got3 = orc.boundary_terms(pb3, orc.PG, [dict(axis=2, hi=True, g_table=tab)], beta=1.0)
    fx, lx = pb3._spans[0]
    fy, ly = pb3._spans[1]
    ax, bx = fx / 4, (lx + 1) / 4
    ay, by = fy / 3, (ly + 1) / 3
    ix = (bx - ax) * (ax + bx) / 2
    iy = (by - ay) * (ay + by) / 2
    face = np.multiply.outer(by - ay, ix) + 10.0 * np.multiply.outer(iy, bx - ax)  # (ry, rx)
    fz, lz = pb3._spans[2]
    want3 = np.multiply.outer((lz == 4).astype(float), face)
    assert np.allclose(got3, want3, rtol=1e-12, atol=1e-14)


def test_dirichlet_rows(orc):
    pb = orc.Problem(2, 2, (4, 3), (3, 3))
    rows = np.arange(np.prod(pb.coef_shape()), dtype=float).reshape(pb.coef_shape()) + 100
    u = -np.ones(pb.coef_shape())
    out = orc.dirichlet_rows(pb, 0b0001 | 0b1000, rows, u)   # x = 0 and y = 1
    want = rows.copy()
    want[:, 0] = -1.0
    want[-1, :] = -1.0
    assert np.array_equal(out, want)
    assert np.array_equal(orc.dirichlet_rows(pb, 0b0010, rows)[:, -1], np.zeros(pb.coef_shape()[0]))


@pytest.mark.parametrize("form", [0, 1, 2])
@pytest.mark.parametrize("p", [2, 3])
def test_mixed_problem_exact_solution(orc, form, p):
    """-Lap u = f, u = 0 on x = 0, du/dn = G elsewhere, with u = x^2 (in the spline
    space, zero on x = 0): f = -2 and G = 2 on x = 1, 0 on y = 0, 1.  The discrete mixed
    system (domain rows with the Laplacian, Neumann rows on x = 1 and y = 0, 1, Dirichlet
    rows on x = 0) holds at u to round-off, in every form (the by-parts form carries its
    own boundary term, so it gets no Neumann flux of u)."""
    ne = (7, 6)
    pb = orc.Problem(2, p, ne, (p + 1, p + 1))
    u = np.tile(quad_coefs(p, ne[0]), (ne[1] + p, 1))
    neu = [dict(axis=0, hi=True, g_const=2.0), dict(axis=1, hi=False), dict(axis=1, hi=True)]
    lhs = -orc.rhs(pb, form, u, 0.0, 1.0, 0.0)
    if form != orc.GALERKIN_BYPARTS:
        lhs = lhs + orc.boundary_terms(pb, form, neu, u, alpha=1.0)
    rhs = orc.rhs(pb, form, None, 0.0, 0.0, 1.0, sin_amp=0.0,
                  f_table=np.full(pb.gauss_shape(), -2.0))
    rhs = rhs + orc.boundary_terms(pb, form, neu, beta=1.0)
    if form != orc.PG:
        lhs = orc.dirichlet_rows(pb, 0b0001, lhs, u)
        rhs = orc.dirichlet_rows(pb, 0b0001, rhs)
        assert np.all(u[:, 0] == 0.0)
    assert np.max(np.abs(lhs - rhs)) < 1e-11 * max(1.0, np.max(np.abs(rhs)))
