"""Exact-rational B-spline integrals on tiny meshes (test-only brute force).

Independent of the oracle: B-splines are built as piecewise polynomials with
``fractions.Fraction`` coefficients, one polynomial per knot interval, and every
integral is taken exactly from antiderivatives -- no quadrature at all.  Used to
pin the oracle's quadrature-based results (exact whenever the Gauss rule is exact
for the integrand's degree).

Polynomials are lists of Fractions, ascending powers of the global coordinate x.
"""
from __future__ import annotations

from fractions import Fraction as F
from functools import lru_cache
from typing import List, Sequence, Tuple

Poly = Tuple[F, ...]


def padd(a: Sequence[F], b: Sequence[F]) -> Poly:
    n = max(len(a), len(b))
    return tuple((a[i] if i < len(a) else F(0)) + (b[i] if i < len(b) else F(0))
                 for i in range(n))


def pscale(a: Sequence[F], s) -> Poly:
    return tuple(c * s for c in a)


def pmul(a: Sequence[F], b: Sequence[F]) -> Poly:
    if not a or not b:
        return ()
    out = [F(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return tuple(out)


def pder(a: Sequence[F]) -> Poly:
    return tuple(i * a[i] for i in range(1, len(a)))


def pint(a: Sequence[F], lo: F, hi: F) -> F:
    """Exact integral of the polynomial a over [lo, hi]."""
    tot = F(0)
    for i, c in enumerate(a):
        tot += c * (hi ** (i + 1) - lo ** (i + 1)) / (i + 1)
    return tot


def peval(a: Sequence[F], x: F) -> F:
    tot = F(0)
    for c in reversed(a):
        tot = tot * x + c
    return tot


class ExactSpace:
    """Open uniform knots on [0, 1] (or [lo, hi]) with ne elements, degree p."""

    def __init__(self, p: int, ne: int, lo=F(0), hi=F(1)):
        self.p, self.ne = p, ne
        self.lo, self.hi = F(lo), F(hi)
        self.h = (self.hi - self.lo) / ne
        self.N = ne + p
        self.t = ([self.lo] * p + [self.lo + k * self.h for k in range(ne + 1)] +
                  [self.hi] * p)
        # pieces[j][e] = polynomial of B_j on element e
        self.pieces = [[self._piece(j, p, e + p) for e in range(ne)] for j in range(self.N)]

    @lru_cache(maxsize=None)
    def _piece(self, j: int, k: int, mu: int) -> Poly:
        """Polynomial of B_{j,k} on knot interval mu (Cox-de Boor on polynomials)."""
        t = self.t
        if k == 0:
            return (F(1),) if j == mu else ()
        out: Poly = ()
        d1 = t[j + k] - t[j]
        d2 = t[j + k + 1] - t[j + 1]
        if d1 != 0:
            out = padd(out, pmul((-t[j] / d1, 1 / d1), self._piece(j, k - 1, mu)))
        if d2 != 0:
            out = padd(out, pmul((t[j + k + 1] / d2, -1 / d2), self._piece(j + 1, k - 1, mu)))
        return out

    def elem(self, e: int) -> Tuple[F, F]:
        return self.lo + e * self.h, self.lo + (e + 1) * self.h

    def piece(self, j: int, e: int, nder: int = 0) -> Poly:
        q = self.pieces[j][e]
        for _ in range(nder):
            q = pder(q)
        return q

    # ---- matrices --------------------------------------------------------
    def gal(self, kind: str) -> List[List[F]]:
        """mass: int B_i B_j; lap: int B_i B_j''; byparts: -int B_i' B_j'."""
        N = self.N
        M = [[F(0)] * N for _ in range(N)]
        for e in range(self.ne):
            a, b = self.elem(e)
            for i in range(e, e + self.p + 1):
                for j in range(e, e + self.p + 1):
                    if kind == "mass":
                        v = pint(pmul(self.piece(i, e), self.piece(j, e)), a, b)
                    elif kind == "lap":
                        v = pint(pmul(self.piece(i, e), self.piece(j, e, 2)), a, b)
                    else:
                        v = -pint(pmul(self.piece(i, e, 1), self.piece(j, e, 1)), a, b)
                    M[i][j] += v
        return M

    def pg(self, kind: str, first: Sequence[int], last: Sequence[int]) -> List[List[F]]:
        """mass: int_{S_r} B_j; lap: int_{S_r} B_j''."""
        M = [[F(0)] * self.N for _ in range(len(first))]
        for r, (s, t) in enumerate(zip(first, last)):
            for e in range(s, t + 1):
                a, b = self.elem(e)
                for j in range(e, e + self.p + 1):
                    M[r][j] += pint(self.piece(j, e, 2 if kind == "lap" else 0), a, b)
        return M

    def weighted(self, j: int, f: Sequence[F]) -> F:
        """int B_j f for a polynomial f."""
        tot = F(0)
        for e in range(max(0, j - self.p), min(self.ne - 1, j) + 1):
            a, b = self.elem(e)
            tot += pint(pmul(self.piece(j, e), f), a, b)
        return tot

    def span_integral(self, s: int, t: int, f: Sequence[F]) -> F:
        a, _ = self.elem(s)
        _, b = self.elem(t)
        return pint(f, a, b)
