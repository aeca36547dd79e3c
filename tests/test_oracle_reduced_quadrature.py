"""Pins of the oracle with the reduced Gauss rule of the Petrov-Galerkin form (CPU only).

Section 4.1 (the scalability test): with piece-wise constant test functions the
integrand of a row is the trial-side function alone, so a right-hand side that is
cubic in each variable needs only 2 Gauss points per axis (exact to degree 3), while
the Galerkin rows multiply it by B_i and need p + 1 points for p = 2 (degree 5).
The same holds for the u-terms: u_h has degree p <= 3 and Lap u_h degree <= p on each
axis, so the 2-point PG rows of alpha u + beta Lap u are exact for p = 2, 3.

Pins (against exact rational integrals, not against the oracle itself):
 * 1D PG mass and Laplacian rows with 2 points equal the exact span integrals
   (support, element and custom spans);
 * the 2-point Galerkin mass rows are NOT exact (degree 2p > 3): the exactness above is
   a property of the PG form, so a PG row that wrongly weighted by B_i would fail;
 * 2D/3D PG rows of alpha u + beta Lap u with 2 points on every axis equal the
   Kronecker combination of the exact 1D rational rows;
 * a separable cubic source given on the 2-point Gauss grid: PG rows equal the exact
   span integrals of the cubic; the Galerkin rows (p = 2) are exact with 3 points and
   not with 2.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from exact_bspline import ExactSpace, pint


def _f(M):
    return np.array([[float(v) for v in row] for row in M])


def _kron_apply(mats, u):
    """Tensor product of per-axis matrices (x, y, z order) applied to u (numpy order)."""
    if len(mats) == 1:
        return mats[0] @ u
    if len(mats) == 2:
        return mats[1] @ u @ mats[0].T
    return np.einsum("zk,yj,xi,kji->zyx", mats[2], mats[1], mats[0], u)


def _normwise(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("p,ne", [(2, 8), (3, 10), (2, 3), (3, 5)])
@pytest.mark.parametrize("spans", ["support", "element", "custom"])
def test_pg_rows_two_points_exact(orc, p, ne, spans):
    if spans == "custom":   # one element short of the support at each end, where possible
        first, last = orc.spans("support", p, ne)
        first = np.minimum(first + 1, last)
    else:
        first, last = orc.spans(spans, p, ne)
    sp = ExactSpace(p, ne)
    PM = orc.matrix_1d(p, ne, 2, orc.MAT_PG_MASS, span=(first, last))
    PD = orc.matrix_1d(p, ne, 2, orc.MAT_PG_LAP, span=(first, last))
    np.testing.assert_allclose(PM, _f(sp.pg("mass", first, last)), atol=1e-15, rtol=0)
    np.testing.assert_allclose(PD, _f(sp.pg("lap", first, last)), atol=1e-12 * ne, rtol=0)


@pytest.mark.parametrize("p,ne", [(2, 8), (3, 10)])
def test_galerkin_two_points_not_exact(orc, p, ne):
    ex = _f(ExactSpace(p, ne).gal("mass"))
    got2 = orc.matrix_1d(p, ne, 2, orc.MAT_GAL_MASS)
    got_full = orc.matrix_1d(p, ne, p + 1, orc.MAT_GAL_MASS)
    assert _normwise(got_full, ex) < 1e-14
    assert _normwise(got2, ex) > 1e-4


CASES = [(1, 2, (9,)), (1, 3, (7,)), (2, 2, (5, 4)), (2, 3, (4, 6)),
         (3, 2, (3, 4, 2)), (3, 3, (2, 3, 4))]


@pytest.mark.parametrize("dim,p,ne", CASES)
def test_pg_u_rows_two_points_equal_exact_kronecker(orc, dim, p, ne):
    pb = orc.Problem(dim=dim, p=p, ne=ne, nq=[2] * dim)
    u = np.random.default_rng(40 + dim).standard_normal(pb.coef_shape())
    ex = []
    for a in range(dim):
        sp = ExactSpace(p, ne[a])
        first, last = orc.spans("support", p, ne[a])
        ex.append((_f(sp.pg("mass", first, last)), _f(sp.pg("lap", first, last))))
    mass = _kron_apply([m for m, _ in ex], u)
    lap = sum(_kron_apply([ex[a][1] if a == t else ex[a][0] for a in range(dim)], u)
              for t in range(dim))
    got_m = orc.rhs(pb, orc.PG, u, alpha=1.0)
    got_l = orc.rhs(pb, orc.PG, u, beta=1.0)
    assert _normwise(got_m, mass) < 1e-13
    assert _normwise(got_l, lap) < 1e-12


def _cubic(rng):
    return [Fr(int(c), 8) for c in rng.integers(-8, 9, size=4)]   # d + c x + b x^2 + a x^3


def _gauss_points(ne, nq):
    xi = np.polynomial.legendre.leggauss(nq)[0]
    return ((np.arange(ne)[:, None] + (xi[None, :] + 1) / 2) / ne).ravel()


def _cubic_table(polys, ne, nq):
    """The separable cubic on the global Gauss grid (numpy order: z, y, x)."""
    vals = []
    for a, q in enumerate(polys):
        x = _gauss_points(ne[a], nq)
        vals.append(sum(float(c) * x ** k for k, c in enumerate(q)))
    out = vals[0]
    for v in vals[1:]:
        out = np.multiply.outer(v, out)
    return out


@pytest.mark.parametrize("dim,p,ne", CASES)
def test_pg_cubic_source_two_points_exact(orc, dim, p, ne):
    rng = np.random.default_rng(50 + dim)
    polys = [_cubic(rng) for _ in range(dim)]
    pb = orc.Problem(dim=dim, p=p, ne=ne, nq=[2] * dim)
    got = orc.rhs(pb, orc.PG, None, gamma=1.0, f_table=_cubic_table(polys, ne, 2))
    per_axis = []
    for a in range(dim):
        sp = ExactSpace(p, ne[a])
        first, last = orc.spans("support", p, ne[a])
        per_axis.append(np.array([float(sp.span_integral(s, t, polys[a]))
                                  for s, t in zip(first, last)]))
    ref = per_axis[0]
    for v in per_axis[1:]:
        ref = np.multiply.outer(v, ref)
    assert _normwise(got, ref) < 1e-13


@pytest.mark.parametrize("ne", [6, 9])
def test_galerkin_cubic_source_needs_three_points(orc, ne):
    """p = 2: int f B_i has degree 5, exact with 3 points and not with 2."""
    p = 2
    polys = [_cubic(np.random.default_rng(60))]
    sp = ExactSpace(p, ne)
    ref = np.array([float(sp.weighted(j, polys[0])) for j in range(ne + p)])
    for nq, exact in ((3, True), (2, False)):
        pb = orc.Problem(dim=1, p=p, ne=(ne,), nq=(nq,))
        got = orc.rhs(pb, orc.GALERKIN_LAPLACIAN, None, gamma=1.0,
                      f_table=_cubic_table(polys, (ne,), nq))
        err = _normwise(got, ref)
        assert (err < 1e-14) if exact else (err > 1e-6), (nq, err)
    # the same source in the PG form with 2 points is exact
    pb = orc.Problem(dim=1, p=p, ne=(ne,), nq=(2,))
    first, last = orc.spans("support", p, ne)
    got = orc.rhs(pb, orc.PG, None, gamma=1.0, f_table=_cubic_table(polys, (ne,), 2))
    ref_pg = np.array([float(pint(polys[0], Fr(s, ne), Fr(t + 1, ne))) for s, t in zip(first, last)])
    assert _normwise(got, ref_pg) < 1e-14
