"""Pins of the oracle's refined-test-space Petrov-Galerkin rows (Section 2: test
B-splines on a refined mesh, summed in sets so that each row's test function is 1 on a
cell and ramps over p refined elements): exact rational integrals on tiny meshes, the
closed-form integral of each test function, the decay of the ramp terms as the test
mesh is refined (the limit is the cell-indicator system), well-posedness of the square
system, the tensor rows against the Kronecker combination of 1D rows, and the
alternating-directions solve against one dense solve."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from exact_bspline import ExactSpace, pint, pmul


def _exact_refined(orc, p, ne, rho, kind):
    """int (sum_{m in J_i} Bhat_m) B_j^{(nder)} exactly, piece by piece (no quadrature)."""
    a, b = orc.refined_cells(p, ne, rho)
    trial = ExactSpace(p, ne)
    test = ExactSpace(p, ne * rho)
    nder = 0 if kind == orc.MAT_PG_MASS else 2
    N = ne + p
    M = [[Fr(0)] * N for _ in range(N)]
    for i in range(N):
        for k in range(ne * rho):                       # refined element k
            lo, hi = Fr(k, ne * rho), Fr(k + 1, ne * rho)
            e = k // rho
            tpoly = ()
            for m in range(max(a[i], k), min(b[i], k + p) + 1):
                piece = test.piece(int(m), k, 0)
                tpoly = tuple((tpoly[q] if q < len(tpoly) else Fr(0)) + (piece[q] if q < len(piece) else Fr(0))
                              for q in range(max(len(tpoly), len(piece))))
            if not tpoly:
                continue
            for j in range(max(0, e), min(N - 1, e + p) + 1):
                M[i][j] += pint(pmul(tpoly, trial.piece(j, e, nder)), lo, hi)
    return np.array([[float(v) for v in row] for row in M])


@pytest.mark.parametrize("p,ne,rho", [(2, 4, 4), (3, 4, 4), (2, 3, 8)])
@pytest.mark.parametrize("kind", [3, 4])
def test_refined_rows_exact(orc, p, ne, rho, kind):
    got = orc.refined_matrix_1d(p, ne, rho, p + 1, kind)
    want = _exact_refined(orc, p, ne, rho, kind)
    scale = np.max(np.abs(want))
    assert np.max(np.abs(got - want)) < 1e-13 * scale


@pytest.mark.parametrize("p,ne,rho", [(2, 9, 4), (3, 7, 8)])
def test_refined_row_sums(orc, p, ne, rho):
    """sum_j int T_i B_j = int T_i (partition of unity of the trial basis) =
    sum_{m in J_i} (that_{m+p+1} - that_m) / (p+1), refined knots in units of the domain."""
    M = orc.refined_matrix_1d(p, ne, rho, p + 1, orc.MAT_PG_MASS)
    a, b = orc.refined_cells(p, ne, rho)
    ns = ne * rho
    t = np.clip(np.arange(ns + 2 * p + 1) - p, 0, ns) / ns
    want = np.array([sum((t[m + p + 1] - t[m]) / (p + 1) for m in range(a[i], b[i] + 1))
                     for i in range(ne + p)])
    assert np.allclose(M.sum(axis=1), want, rtol=1e-13, atol=0)
    # and the Laplacian rows sum to 0 (the operator kills constants)
    L = orc.refined_matrix_1d(p, ne, rho, p + 1, orc.MAT_PG_LAP)
    assert np.max(np.abs(L.sum(axis=1))) < 1e-10 * np.max(np.abs(L))


def test_ramp_terms_decay_with_refinement(orc):
    """p = 2: the cells are the Greville-midpoint cells exactly for rho = 4, 8, 16, 32 (the
    midpoints are at 1/4 and at integers), and the rows tend to the cell integrals
    int_{cell_i} B_j as the ramps (p refined elements wide) shrink: halving rho's ramp
    halves the difference."""
    p, ne = 2, 6
    trial = ExactSpace(p, ne)
    cuts = [Fr(0), Fr(1, 4)] + [Fr(k) for k in range(1, ne)] + [Fr(ne) - Fr(1, 4), Fr(ne)]
    N = ne + p
    Mc = np.zeros((N, N))
    for i in range(N):
        x0, x1 = cuts[i] / ne, cuts[i + 1] / ne
        for e in range(ne):
            lo, hi = max(x0, Fr(e, ne)), min(x1, Fr(e + 1, ne))
            if lo >= hi:
                continue
            for j in range(e, e + p + 1):
                Mc[i, j] += float(pint(trial.piece(j, e, 0), lo, hi))
    errs = []
    for rho in (4, 8, 16, 32):
        a, b = orc.refined_cells(p, ne, rho)
        assert np.array_equal(a, [int(c * rho) for c in cuts[:-1]])
        errs.append(np.max(np.abs(orc.refined_matrix_1d(p, ne, rho, 3, orc.MAT_PG_MASS) - Mc)))
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    assert all(1.7 < r < 2.3 for r in ratios), (errs, ratios)


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("ne,rho", [(8, 4), (32, 4), (32, 8)])
def test_refined_system_is_regular(orc, p, ne, rho):
    """Square and well conditioned, unlike the singular system of whole-element spans."""
    M = orc.refined_matrix_1d(p, ne, rho, p + 1, orc.MAT_PG_MASS)
    assert np.linalg.cond(M) < 200.0
    # every row's columns lie in the window r-p .. r+p of the banded layout
    for i in range(ne + p):
        nz = np.nonzero(np.abs(M[i]) > 0)[0]
        assert nz.min() >= i - p and nz.max() <= i + p


@pytest.mark.parametrize("dim,p,ne,rho", [(2, 2, (5, 4), (4, 8)), (3, 3, (3, 4, 2), (4, 4, 8))])
def test_refined_tensor_rows_are_kronecker(orc, dim, p, ne, rho):
    """The tensor rows, evaluated point by point on the sub-element Gauss grid, equal the
    Kronecker combination of the 1D rows: mass (x) ... and sum_t D_t (x) mass_others."""
    pb = orc.Problem(dim, p, ne, [p + 1] * dim)
    u = np.random.default_rng(51).standard_normal(pb.coef_shape())
    got = orc.refined_rhs(pb, rho, u, alpha=0.6, beta=-1.1)
    Ms = [orc.refined_matrix_1d(p, ne[a], rho[a], p + 1, orc.MAT_PG_MASS) for a in range(dim)]
    Ds = [orc.refined_matrix_1d(p, ne[a], rho[a], p + 1, orc.MAT_PG_LAP) for a in range(dim)]

    def kron(mats):
        K = np.ones((1, 1))
        for a in reversed(range(dim)):
            K = np.kron(K, mats[a])
        return K
    want = 0.6 * kron(Ms) @ u.ravel()
    for t in range(dim):
        want = want - 1.1 * kron([Ds[a] if a == t else Ms[a] for a in range(dim)]) @ u.ravel()
    assert np.max(np.abs(got.ravel() - want)) < 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("dim,p,ne,rho", [(2, 3, (6, 5), (4, 4)), (3, 2, (4, 3, 5), (8, 4, 4))])
def test_refined_solve_equals_dense(orc, dim, p, ne, rho):
    pb = orc.Problem(dim, p, ne, [p + 1] * dim)
    b = np.random.default_rng(52).standard_normal(pb.coef_shape())
    K = np.ones((1, 1))
    for a in reversed(range(dim)):
        K = np.kron(K, orc.refined_matrix_1d(p, ne[a], rho[a], p + 1, orc.MAT_PG_MASS))
    want = np.linalg.solve(K, b.ravel()).reshape(b.shape)
    got = orc.refined_solve(pb, rho, b)
    assert np.max(np.abs(got - want)) < 1e-11 * np.max(np.abs(want))
