"""Pins of the oracle's B-spline basis and Gauss rule (CPU only).

Basis: the paper's worked example (Section 2), partition of unity at every Gauss
point (Section 2, "black terms"), the B-spline count of every timing table, and
agreement with an independent exact-rational construction and with scipy's
B-spline evaluator.  Quadrature: exactness degree 2n-1 of the n-point rule
(Section 4.1 reduced-quadrature argument) and agreement with numpy's
Gauss-Legendre routine.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from exact_bspline import ExactSpace, peval

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_example():
    sup = {}
    with open(os.path.join(GOLDEN, "paper_example_supports.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            k, *v = line.split()
            if k.startswith("B"):
                sup[int(k[1:])] = (int(v[0]), int(v[1]))
            elif k == "degree":
                p = int(v[0])
            elif k == "elements":
                ne = int(v[0])
            elif k == "knots":
                knots = [int(x) for x in v]
    return p, ne, knots, sup


def test_paper_example_supports(orc):
    """P1: supports of the 7 quadratic B-splines on [0 0 0 1 2 3 4 5 5 5]."""
    p, ne, knots, printed = _read_example()
    assert len(knots) == ne + 2 * p + 1 and len(printed) == ne + p
    # reading of the two printed entries that contradict the knot vector
    reading = dict(printed)
    reading[5] = (knots[4], knots[7])
    reading[6] = (knots[5], knots[8])
    assert reading[5] == (2, 5) and reading[6] == (3, 5)
    # mirror symmetry of the open uniform knot vector: B_i <-> B_{N+1-i}
    for i in range(1, ne + p + 1):
        a, b = reading[i]
        c, d = reading[ne + p + 1 - i]
        assert (a, b) == (ne - d, ne - c)
    # the printed entries other than the two typos agree with the knot rule
    for i in (1, 2, 3, 4, 7):
        assert printed[i] == (knots[i - 1], knots[i + 2])
    # oracle: B_j is nonzero exactly on the elements inside its support
    for j in range(1, ne + p + 1):
        a, b = reading[j]
        for e in range(ne):
            B = orc.basis_eval(p, ne, e + 0.5, lo=0.0, hi=float(ne), nder=0)[0]
            inside = a <= e and e + 1 <= b
            assert (abs(B[j - 1]) > 1e-12) == inside, (j, e)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("ne", [1, 2, 5, 13])
def test_partition_of_unity_at_gauss_points(orc, p, ne):
    """P2: sum_j B_j = 1, sum_j B_j' = 0, sum_j B_j'' = 0 at every Gauss point."""
    lo, hi = -0.3, 1.7
    h = (hi - lo) / ne
    for nq in (2, 3, 4):
        xi, _ = orc.gauss_legendre(nq)
        for e in range(ne):
            for q in range(nq):
                x = lo + (e + (xi[q] + 1) / 2) * h
                B = orc.basis_eval(p, ne, x, lo=lo, hi=hi, nder=2)
                assert abs(B[0].sum() - 1.0) <= 4e-16 * (p + 1)
                assert abs(B[1].sum()) <= 1e-13 / h
                assert abs(B[2].sum()) <= 1e-12 / h ** 2
                # exactly p+1 nonzero functions, those of element e
                nz = np.nonzero(np.abs(B[0]) > 0)[0]
                assert list(nz) == list(range(e, e + p + 1))
                assert np.all(B[0] >= 0)


def test_nrdof_of_every_table(orc):
    """P3: the #NRDOF column of Tables 1, 1a, 2 is (n+p)^d with N = n+p B-splines per axis."""
    rows = []
    with open(os.path.join(GOLDEN, "nrdof_tables.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                t, d, p, n, nr = line.split()
                rows.append((t, int(d), int(p), int(n), int(nr)))
    assert len(rows) == 18
    for _, d, p, n, nrdof in rows:
        nb = orc.basis_eval(p, n, 0.5, nder=0).shape[1]
        assert nb ** d == nrdof


@pytest.mark.parametrize("p,ne", [(2, 5), (3, 7), (4, 4)])
def test_basis_matches_exact_rational(orc, p, ne):
    """Oracle values and derivatives equal the exact piecewise polynomials."""
    sp = ExactSpace(p, ne)
    rng = np.random.default_rng(0)
    for _ in range(40):
        x = Fraction(int(rng.integers(0, 10**6)), 10**6)
        e = min(int(x * ne), ne - 1)
        B = orc.basis_eval(p, ne, float(x), nder=2)
        for j in range(ne + p):
            for d in range(3):
                ex = peval(sp.piece(j, e, d), x) if e <= j <= e + p else 0
                assert abs(B[d, j] - float(ex)) <= 1e-12 * max(1.0, ne ** d)


@pytest.mark.parametrize("p,ne", [(2, 6), (3, 9)])
def test_basis_matches_scipy(orc, p, ne):
    """Oracle values and derivatives equal scipy.interpolate.BSpline on the same knots."""
    from scipy.interpolate import BSpline
    t = np.concatenate([np.zeros(p), np.linspace(0, 1, ne + 1), np.ones(p)])
    xs = np.linspace(0.0, 1.0, 57)[1:-1]
    for j in range(ne + p):
        c = np.zeros(ne + p)
        c[j] = 1.0
        s = BSpline(t, c, p)
        for d in range(3):
            ref = s.derivative(d)(xs) if d else s(xs)
            ours = np.array([orc.basis_eval(p, ne, x, nder=2)[d, j] for x in xs])
            np.testing.assert_allclose(ours, ref, atol=1e-11 * ne ** d, rtol=0)


@pytest.mark.parametrize("n", range(1, 11))
def test_gauss_exactness(orc, n):
    """P4: the n-point rule integrates x^k exactly for k <= 2n-1 and not for k = 2n."""
    xi, w = orc.gauss_legendre(n)
    assert np.all(np.diff(xi) > 0)
    for k in range(2 * n + 1):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        got = float(np.sum(w * xi ** k))
        if k <= 2 * n - 1:
            assert abs(got - exact) < 1e-14
        else:
            assert abs(got - exact) > 1e-6


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 20])
def test_gauss_matches_numpy(orc, n):
    xi, w = orc.gauss_legendre(n)
    rx, rw = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(xi, rx, atol=1e-15)
    np.testing.assert_allclose(w, rw, atol=1e-15)
