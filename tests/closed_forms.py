"""Closed forms from B-spline theory used as pins at any size (independent of the oracle
and of the library): quadratic precision of B-splines on open uniform knots, and the
exact integrals of the reproduced polynomial over support spans."""
import numpy as np


def knots(p, ne, lo=0.0, hi=1.0):
    inner = lo + (hi - lo) * np.arange(ne + 1) / ne
    return np.concatenate([np.full(p, lo), inner, np.full(p, hi)])


def quad_coefs(p, ne):
    """Coefficients c_j with sum_j c_j B_j(x) = x^2 on [0, 1]: the blossom of x^2 at the
    knots t_{j+1} .. t_{j+p}, i.e. the mean of t_a t_b over the pairs a < b."""
    t = knots(p, ne)
    k = np.stack([t[i + 1:i + 1 + ne + p] for i in range(p)])
    pairs = (k.sum(axis=0) ** 2 - (k * k).sum(axis=0)) / 2.0
    return pairs / (p * (p - 1) / 2.0)


def bspline_integrals(p, ne):
    """int B_j over [0, 1]: (t_{j+p+1} - t_j) / (p + 1)."""
    t = knots(p, ne)
    return (t[p + 1:p + 1 + ne + p] - t[:ne + p]) / (p + 1)


def support_span_moments(p, ne, rows):
    """|S_r| and int_{S_r} x^2 dx for S_r = supp B_r, without cancellation: the width comes
    from the element counts and int_a^b x^2 = (b - a)(a^2 + ab + b^2)/3."""
    rows = np.asarray(rows)
    s = np.maximum(rows - p, 0)
    t = np.minimum(rows, ne - 1)
    a, b = s / ne, (t + 1) / ne
    width = (t + 1 - s) / ne
    return width, width * (a * a + a * b + b * b) / 3.0


def lin_coefs(p, ne):
    """Coefficients c_j with sum_j c_j B_j(x) = x on [0, 1]: the Greville abscissae, the
    mean of the knots t_{j+1} .. t_{j+p}."""
    t = knots(p, ne)
    return np.mean(np.stack([t[i + 1:i + 1 + ne + p] for i in range(p)]), axis=0)
