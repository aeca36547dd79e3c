"""Pins of the oracle's 1D system matrices (CPU only).

 * classical uniform-knot stencils of the quadratic B-spline mass and stiffness
   matrices (closed forms), and exact-rational integrals for p = 2, 3;
 * Petrov-Galerkin rows: every row of int_{S_r} B_j sums to |S_r| (partition of
   unity) and every row of int_{S_r} B_j'' sums to 0;
 * Laplacian form minus by-parts form equals the boundary matrix
   B_i(1) B_j'(1) - B_i(0) B_j'(0) (Section 1: the two agree for test functions
   that vanish on the boundary);
 * the row-sum identity of Section 2: the sum of the Galerkin rows of the p+m
   B-splines that are nonzero on a span equals the Petrov-Galerkin row of that
   span plus the ramp ("red"/"blue") terms on the p elements beyond each end.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from exact_bspline import ExactSpace, padd, pint, pmul


def _f(M):
    return np.array([[float(v) for v in row] for row in M])


@pytest.mark.parametrize("ne", [8, 11])
def test_quadratic_closed_form_stencils(orc, ne):
    """P5/P6: interior rows for uniform quadratic B-splines, 3-point Gauss.
    stiffness int B_i'B_j' = (1/h)[-1/6, -1/3, 1, -1/3, -1/6];
    mass int B_i B_j = h[1/120, 13/60, 11/20, 13/60, 1/120]."""
    h = 1.0 / ne
    K = orc.matrix_1d(2, ne, 3, orc.MAT_GAL_BYPARTS)
    M = orc.matrix_1d(2, ne, 3, orc.MAT_GAL_MASS)
    KL = orc.matrix_1d(2, ne, 3, orc.MAT_GAL_LAP)
    stiff = np.array([-1 / 6, -1 / 3, 1.0, -1 / 3, -1 / 6]) / h
    mass = np.array([1 / 120, 13 / 60, 11 / 20, 13 / 60, 1 / 120]) * h
    for r in range(4, ne - 2):
        np.testing.assert_allclose(-K[r, r - 2:r + 3], stiff, rtol=1e-13, atol=1e-13 / h)
        np.testing.assert_allclose(-KL[r, r - 2:r + 3], stiff, rtol=1e-13, atol=1e-12 / h)
        np.testing.assert_allclose(M[r, r - 2:r + 3], mass, rtol=1e-13)
        assert np.all(K[r, :r - 2] == 0) and np.all(K[r, r + 3:] == 0)


@pytest.mark.parametrize("p,ne", [(2, 8), (3, 10)])
@pytest.mark.parametrize("kind,name", [(0, "mass"), (1, "lap"), (2, "byparts")])
def test_galerkin_equals_exact(orc, p, ne, kind, name):
    """P5/P6/P12: (p+1)-point Gauss integrates these products exactly."""
    ex = _f(ExactSpace(p, ne).gal(name))
    got = orc.matrix_1d(p, ne, p + 1, kind)
    np.testing.assert_allclose(got, ex, atol=1e-13 * ne ** 2, rtol=0)


@pytest.mark.parametrize("p,ne", [(2, 8), (3, 10), (2, 3), (3, 4)])
@pytest.mark.parametrize("spans", ["support", "element"])
def test_pg_equals_exact_and_row_sums(orc, p, ne, spans):
    """P7/P8: Petrov-Galerkin mass and Laplacian rows, exact; row sums |S_r| and 0."""
    first, last = orc.spans(spans, p, ne)
    sp = ExactSpace(p, ne)
    h = 1.0 / ne
    PM = orc.matrix_1d(p, ne, p + 1, orc.MAT_PG_MASS, span=(first, last))
    PD = orc.matrix_1d(p, ne, p + 1, orc.MAT_PG_LAP, span=(first, last))
    np.testing.assert_allclose(PM, _f(sp.pg("mass", first, last)), atol=1e-15, rtol=0)
    np.testing.assert_allclose(PD, _f(sp.pg("lap", first, last)), atol=1e-12 * ne, rtol=0)
    np.testing.assert_allclose(PM.sum(axis=1), (last - first + 1) * h, rtol=1e-14)
    np.testing.assert_allclose(PD.sum(axis=1), 0.0, atol=1e-12 * ne)


def test_pg_interior_stencils(orc):
    """P7/P8 interior rows with support spans (exact rationals, verified above):
    p=2 mass h[1/6,5/6,1,5/6,1/6], Lap (1/h)[1,-1,0,-1,1];
    p=3 mass h[1/24,1/2,23/24,1,23/24,1/2,1/24], Lap (1/h)[1/2,0,-1/2,0,-1/2,0,1/2]."""
    ne = 16
    h = 1.0 / ne
    cases = {2: ([1 / 6, 5 / 6, 1, 5 / 6, 1 / 6], [1, -1, 0, -1, 1]),
             3: ([1 / 24, 1 / 2, 23 / 24, 1, 23 / 24, 1 / 2, 1 / 24],
                 [0.5, 0, -0.5, 0, -0.5, 0, 0.5])}
    for p, (m, d) in cases.items():
        PM = orc.matrix_1d(p, ne, p + 1, orc.MAT_PG_MASS)
        PD = orc.matrix_1d(p, ne, p + 1, orc.MAT_PG_LAP)
        r = ne // 2
        np.testing.assert_allclose(PM[r, r - p:r + p + 1], np.array(m) * h, atol=1e-15)
        np.testing.assert_allclose(PD[r, r - p:r + p + 1], np.array(d) / h, atol=1e-11)


@pytest.mark.parametrize("p,ne", [(2, 6), (3, 9), (2, 12)])
def test_laplacian_minus_byparts_is_boundary_matrix(orc, p, ne):
    """P10: int B_i B_j'' - (-int B_i'B_j') = B_i(1)B_j'(1) - B_i(0)B_j'(0)."""
    KL = orc.matrix_1d(p, ne, p + 1, orc.MAT_GAL_LAP)
    KB = orc.matrix_1d(p, ne, p + 1, orc.MAT_GAL_BYPARTS)
    B0 = orc.basis_eval(p, ne, 0.0, nder=1)
    B1 = orc.basis_eval(p, ne, 1.0, nder=1)
    bnd = np.outer(B1[0], B1[1]) - np.outer(B0[0], B0[1])
    np.testing.assert_allclose(KL - KB, bnd, atol=1e-12 * ne)
    # the boundary matrix lives in the first and the last row only
    assert np.all(bnd[1:-1] == 0)
    h = 1.0 / ne
    np.testing.assert_allclose(bnd[0, :2], [p / h, -p / h], rtol=1e-13)
    np.testing.assert_allclose(bnd[-1, -2:], [-p / h, p / h], rtol=1e-13)


def _ramps(sp: ExactSpace, s, t, op_order):
    """R(S, j): integral over the ramp elements of (sum_{m in J(S)} B_m) * op(B_j)."""
    p, ne = sp.p, sp.ne
    J = range(s, min(t + p, sp.N - 1) + 1)
    R = [Fr(0)] * sp.N
    for e in list(range(max(0, s - p), s)) + list(range(t + 1, min(ne - 1, t + p) + 1)):
        a, b = sp.elem(e)
        test = ()
        for m in J:
            if e <= m <= e + p:
                test = padd(test, sp.piece(m, e))
        for j in range(e, e + p + 1):
            R[j] += pint(pmul(test, sp.piece(j, e, op_order)), a, b)
    return R


@pytest.mark.parametrize("p,ne", [(2, 5), (2, 9), (3, 10)])
@pytest.mark.parametrize("spans", ["support", "element", "custom"])
def test_row_sum_identity(orc, p, ne, spans):
    """P-ID (Section 2): PG row of span S = sum of the Galerkin rows J(S) = [s, t+p]
    minus the ramp terms; exact for any quadrature because B-splines sum to one
    pointwise.  Here with the Laplacian form and the mass, 2-point and (p+1)-point Gauss."""
    if spans == "custom":
        first = np.array([0, 1, 2, 0, ne - 3], dtype=np.int64)
        last = np.array([0, 3, ne - 1, ne - 1, ne - 2], dtype=np.int64)
    else:
        first, last = orc.spans(spans, p, ne)
    sp = ExactSpace(p, ne)
    for nq in (2, p + 1):
        for op, gk, pk in ((0, orc.MAT_GAL_MASS, orc.MAT_PG_MASS),
                           (2, orc.MAT_GAL_LAP, orc.MAT_PG_LAP)):
            G = orc.matrix_1d(p, ne, nq, gk)
            P = orc.matrix_1d(p, ne, nq, pk, span=(first, last))
            for r, (s, t) in enumerate(zip(first, last)):
                rows = G[s:min(t + p, ne + p - 1) + 1].sum(axis=0)
                if nq == p + 1:   # ramps exact for the (p+1)-point rule
                    R = np.array([float(v) for v in _ramps(sp, int(s), int(t), op)])
                    np.testing.assert_allclose(P[r], rows - R, atol=1e-12 * ne ** 2)
                if s == 0 and t == ne - 1:   # whole domain: no ramps
                    np.testing.assert_allclose(P[r], rows, atol=1e-12 * ne ** 2)
