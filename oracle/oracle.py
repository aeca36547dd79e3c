"""ctypes/numpy front end of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It loads ``oracle/liboracle.so`` (plain C,
built by ``oracle/build.py``) and shares no code with the GPU library.

Axis order is (x, y, z) in every per-axis argument; numpy arrays are C-ordered
(N_z, N_y, N_x), x fastest.  Definitions follow arXiv:1910.08535: Section 2 for
the basis and the row sums, Section 3 for the tensor product, Section 4.1 for the
generation loops and the alternating-directions solve with the Galerkin mass,
Section 4.2 for the explicit steps.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

GALERKIN_BYPARTS, GALERKIN_LAPLACIAN, PG = 0, 1, 2
MAT_GAL_MASS, MAT_GAL_LAP, MAT_GAL_BYPARTS, MAT_PG_MASS, MAT_PG_LAP = 0, 1, 2, 3, 4

_PL = C.POINTER(C.c_long)
_PD = C.POINTER(C.c_double)


class _Problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("p", C.c_int), ("ne", C.c_long * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("nq", C.c_int * 3),
                ("nspan", C.c_long * 3), ("span_first", _PL * 3), ("span_last", _PL * 3)]


class _Source(C.Structure):
    _fields_ = [("table", _PD), ("sin_amp", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # type: ignore
            _b.build()
        L = C.CDLL(LIB_PATH)
        L.or_gauss_legendre.argtypes = [C.c_int, _PD, _PD]
        L.or_basis_eval.argtypes = [C.c_int, C.c_long, C.c_double, C.c_double, C.c_double,
                                    C.c_int, _PD]
        L.or_matrix_1d.argtypes = [C.c_int, C.c_long, C.c_double, C.c_double, C.c_int, C.c_int,
                                   C.c_long, _PL, _PL, _PD]
        L.or_rhs.argtypes = [C.POINTER(_Problem), C.c_int, _PD, C.c_double, C.c_double,
                             C.c_double, C.POINTER(_Source), C.c_long, C.c_long, _PD]
        L.or_explicit_step.argtypes = [C.POINTER(_Problem), _PD, C.c_double,
                                       C.POINTER(_Source), C.c_int]
        L.or_num_threads.argtypes = []
        for fn in (L.or_gauss_legendre, L.or_basis_eval, L.or_matrix_1d, L.or_rhs,
                   L.or_explicit_step, L.or_num_threads):
            fn.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_PD)


def _lp(a: np.ndarray):
    return a.ctypes.data_as(_PL)


def num_threads() -> int:
    return int(lib().or_num_threads())


def gauss_legendre(nq: int) -> Tuple[np.ndarray, np.ndarray]:
    xi = np.zeros(nq)
    w = np.zeros(nq)
    if lib().or_gauss_legendre(nq, _dp(xi), _dp(w)):
        raise ValueError("bad nq")
    return xi, w


def basis_eval(p: int, ne: int, x: float, lo: float = 0.0, hi: float = 1.0,
               nder: int = 2) -> np.ndarray:
    """All N = ne + p B-splines and their derivatives at x, shape (nder+1, N)."""
    out = np.zeros((nder + 1) * (ne + p))
    if lib().or_basis_eval(p, ne, lo, hi, float(x), nder, _dp(out)):
        raise ValueError("bad basis arguments")
    return out.reshape(nder + 1, ne + p)


def spans(kind: str, p: int, ne: int) -> Tuple[np.ndarray, np.ndarray]:
    """Test spans along one axis (inclusive element ranges).

    ``support``: row r in [0, ne+p) takes S_r = supp B_r = [max(0, r-p), min(ne-1, r)],
    i.e. every element's integral is added to the p+1 rows of the B-splines
    that live on it, as in the piece-wise-constant generation loop of Section 4.1.
    ``element``: row e in [0, ne) takes S_e = {e}, the single-element integrals
    (the example's rows where p+1 consecutive B-splines sum to one, Section 2).
    """
    if kind == "support":
        r = np.arange(ne + p)
        return (np.maximum(0, r - p).astype(np.int64), np.minimum(ne - 1, r).astype(np.int64))
    if kind == "element":
        r = np.arange(ne, dtype=np.int64)
        return r.copy(), r.copy()
    raise ValueError(kind)


def matrix_1d(p: int, ne: int, nq: int, kind: int, lo: float = 0.0, hi: float = 1.0,
              span: Optional[Tuple[np.ndarray, np.ndarray]] = None) -> np.ndarray:
    N = ne + p
    if kind in (MAT_PG_MASS, MAT_PG_LAP):
        if span is None:
            span = spans("support", p, ne)
        first = np.ascontiguousarray(span[0], dtype=np.int64)
        last = np.ascontiguousarray(span[1], dtype=np.int64)
        nrows = len(first)
    else:
        first = last = np.zeros(1, dtype=np.int64)
        nrows = N
    out = np.zeros(nrows * N)
    rc = lib().or_matrix_1d(p, ne, lo, hi, nq, kind, nrows, _lp(first), _lp(last), _dp(out))
    if rc:
        raise ValueError(f"or_matrix_1d failed ({rc})")
    return out.reshape(nrows, N)


@dataclass
class Problem:
    """A tensor-product B-spline space with its Gauss rule and test spans."""
    dim: int
    p: int
    ne: Sequence[int]
    nq: Sequence[int]
    lo: Sequence[float] = (0.0, 0.0, 0.0)
    hi: Sequence[float] = (1.0, 1.0, 1.0)
    span_kind: str = "support"
    custom_spans: Optional[Sequence[Tuple[np.ndarray, np.ndarray]]] = None
    _spans: list = field(default_factory=list, repr=False)

    def __post_init__(self):
        self.ne = tuple(int(v) for v in self.ne)[: self.dim]
        self.nq = tuple(int(v) for v in self.nq)[: self.dim]
        if self.custom_spans is not None:
            self._spans = [(np.ascontiguousarray(f, dtype=np.int64),
                            np.ascontiguousarray(l, dtype=np.int64))
                           for f, l in self.custom_spans]
        else:
            self._spans = [spans(self.span_kind, self.p, n) for n in self.ne]

    @property
    def nbasis(self) -> Tuple[int, ...]:
        return tuple(n + self.p for n in self.ne)

    @property
    def nspan(self) -> Tuple[int, ...]:
        return tuple(len(s[0]) for s in self._spans)

    def shape(self, form: int) -> Tuple[int, ...]:
        per_axis = self.nspan if form == PG else self.nbasis
        return tuple(reversed(per_axis))

    def coef_shape(self) -> Tuple[int, ...]:
        return tuple(reversed(self.nbasis))

    def gauss_shape(self) -> Tuple[int, ...]:
        return tuple(reversed([n * q for n, q in zip(self.ne, self.nq)]))

    def _struct(self) -> _Problem:
        s = _Problem()
        s.dim = self.dim
        s.p = self.p
        for a in range(3):
            real = a < self.dim
            s.ne[a] = self.ne[a] if real else 1
            s.lo[a] = self.lo[a] if real else 0.0
            s.hi[a] = self.hi[a] if real else 1.0
            s.nq[a] = self.nq[a] if real else 1
            if real:
                f, l = self._spans[a]
                s.nspan[a] = len(f)
                s.span_first[a] = _lp(f)
                s.span_last[a] = _lp(l)
            else:
                s.nspan[a] = 1
        return s


def _source(table: Optional[np.ndarray], sin_amp: float):
    src = _Source()
    src.table = _dp(table) if table is not None else None
    src.sin_amp = float(sin_amp)
    return src


def rhs(pb: Problem, form: int, u: Optional[np.ndarray], alpha: float = 0.0, beta: float = 0.0,
        gamma: float = 0.0, f_table: Optional[np.ndarray] = None, sin_amp: float = 0.0,
        rows: Optional[Tuple[int, int]] = None) -> np.ndarray:
    """b = int T_r (alpha u_h + beta Lap u_h + gamma f) for every row r.

    T_r = B_r (Galerkin; the by-parts form integrates the Laplacian term by
    parts) or the indicator of the span S_r (PG).  ``rows`` restricts the output
    to a slab [r0, r1) of the outermost axis."""
    shape = pb.shape(form)
    if u is not None:
        u = np.ascontiguousarray(u, dtype=np.float64)
        assert u.shape == pb.coef_shape(), (u.shape, pb.coef_shape())
    if f_table is not None:
        f_table = np.ascontiguousarray(f_table, dtype=np.float64)
        assert f_table.shape == pb.gauss_shape()
    r0, r1 = (0, shape[0]) if rows is None else rows
    out = np.zeros((r1 - r0,) + shape[1:])
    st = pb._struct()
    src = _source(f_table, sin_amp)
    rc = lib().or_rhs(C.byref(st), form, _dp(u), alpha, beta, gamma, C.byref(src), r0, r1,
                      _dp(out))
    if rc:
        raise ValueError(f"or_rhs failed ({rc})")
    return out


def explicit_step(pb: Problem, u: np.ndarray, dt: float, f_table: Optional[np.ndarray] = None,
                  sin_amp: float = 0.0, nsteps: int = 1) -> np.ndarray:
    """nsteps forward-Euler steps, PG form, lumped left-hand side (returns a copy)."""
    v = np.array(u, dtype=np.float64, copy=True, order="C")
    assert v.shape == pb.coef_shape()
    if f_table is not None:
        f_table = np.ascontiguousarray(f_table, dtype=np.float64)
    st = pb._struct()
    src = _source(f_table, sin_amp)
    rc = lib().or_explicit_step(C.byref(st), _dp(v), dt, C.byref(src), nsteps)
    if rc:
        raise ValueError(f"or_explicit_step failed ({rc})")
    return v


def span_lengths(pb: Problem) -> Tuple[np.ndarray, ...]:
    """Per-axis knot lengths |S_r| of the test spans (uniform knots)."""
    out = []
    for a in range(pb.dim):
        h = (pb.hi[a] - pb.lo[a]) / pb.ne[a]
        f, l = pb._spans[a]
        out.append((l - f + 1) * h)
    return tuple(out)


def galerkin_mass_1d(pb: Problem, a: int) -> np.ndarray:
    """Dense 1D Galerkin mass matrix M_a(i, j) = int B_i B_j of axis a (Section 4.1)."""
    return matrix_1d(pb.p, pb.ne[a], pb.nq[a], MAT_GAL_MASS, pb.lo[a], pb.hi[a])


def ads_solve(pb: Problem, b: np.ndarray) -> np.ndarray:
    """Solves (M_z (x) M_y (x) M_x) x = b, x fastest, with M_a the 1D Galerkin mass.

    The alternating-directions direct solver of Section 4.1: the Kronecker structure
    turns the solve into three families of 1D systems with many right-hand sides,
    first along x (one right-hand side per (y, z) line), then along y, then along z.
    Each family is one call of numpy.linalg.solve (dense LU with partial pivoting)
    on all of its lines at once."""
    x = np.array(b, dtype=np.float64, copy=True)
    assert x.shape == pb.coef_shape(), (x.shape, pb.coef_shape())
    for a in range(pb.dim):
        M = galerkin_mass_1d(pb, a)
        ax = pb.dim - 1 - a                      # numpy axis of mesh axis a
        lines = np.moveaxis(x, ax, 0)
        sol = np.linalg.solve(M, lines.reshape(M.shape[0], -1))
        x = np.moveaxis(sol.reshape(lines.shape), 0, ax)
    return np.ascontiguousarray(x)


def galerkin_step(pb: Problem, u: np.ndarray, dt: float, form: int = GALERKIN_LAPLACIAN,
                  f_table: Optional[np.ndarray] = None, sin_amp: float = 0.0,
                  nsteps: int = 1) -> np.ndarray:
    """nsteps forward-Euler steps of u_t = Lap u + f in a Galerkin form with the
    consistent mass (Section 4.2): M u_{t+1} = int B_r (u_t + dt Lap u_t + dt f), the
    right-hand side generated as in the projection problem and the mass system solved
    with the alternating-directions solver."""
    v = np.array(u, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        b = rhs(pb, form, v, 1.0, dt, dt, f_table, sin_amp)
        v = ads_solve(pb, b)
    return v


def boundary_terms(pb: Problem, form: int, sides, u: Optional[np.ndarray] = None,
                   alpha: float = 0.0, beta: float = 0.0) -> np.ndarray:
    """Boundary rows of the problem with Neumann conditions (Section 4.3):

        b_r = sum over the listed sides G of  int_G T_r (alpha du_h/dn + beta G) dS,

    T_r = B_r (Galerkin forms) or the indicator of the span S_r (PG), n the outward
    normal.  ``sides`` lists dicts {"axis": a, "hi": bool, "g_table": array or None,
    "g_const": float}; a side's table holds G at its Gauss points, tangential axes in
    increasing order with the first fastest (numpy shape reversed).  Evaluated point by
    point: the side's Gauss points, the basis at each of them and at the side's
    coordinate, and the test function's value there."""
    dim, p = pb.dim, pb.p
    shape = pb.shape(form)
    out = np.zeros(shape)
    if u is not None:
        u = np.asarray(u, dtype=np.float64)
        assert u.shape == pb.coef_shape()
    for sd in sides:
        a, hi = int(sd["axis"]), bool(sd["hi"])
        xs = pb.hi[a] if hi else pb.lo[a]
        nrm = 1.0 if hi else -1.0
        Ba = basis_eval(p, pb.ne[a], xs, pb.lo[a], pb.hi[a], nder=1)
        # normal factor of each row: PG = does the span reach the side; Galerkin = B_r(side)
        if form == PG:
            f, l = pb._spans[a]
            wa = ((l == pb.ne[a] - 1) if hi else (f == 0)).astype(np.float64)
        else:
            wa = Ba[0].copy()
        tang = [b for b in range(dim) if b != a]
        # Gauss points of the side, per tangential axis: weights, elements, basis values
        Tb, Bb = [], []
        for b in tang:
            xi, w = gauss_legendre(pb.nq[b])
            hb = (pb.hi[b] - pb.lo[b]) / pb.ne[b]
            e = np.repeat(np.arange(pb.ne[b]), pb.nq[b])
            xq = pb.lo[b] + hb * (e + (np.tile(xi, pb.ne[b]) + 1.0) / 2.0)
            wq = np.tile(w, pb.ne[b]) * hb / 2.0
            vals = np.stack([basis_eval(p, pb.ne[b], x, pb.lo[b], pb.hi[b], nder=0)[0] for x in xq])
            Bb.append(vals)                                     # (points, N_b)
            if form == PG:
                fb, lb = pb._spans[b]
                ind = (e[None, :] >= fb[:, None]) & (e[None, :] <= lb[:, None])
                Tb.append(ind * wq[None, :])                    # (R_b, points)
            else:
                Tb.append(vals.T * wq[None, :])                 # (N_b, points)
        # integrand at the side's points (numpy order: tangential axes reversed)
        val = np.zeros(tuple(len(B) for B in reversed(Bb)))
        if u is not None and alpha != 0.0:
            dn = np.moveaxis(u, dim - 1 - a, 0)
            dn = nrm * np.tensordot(Ba[1], dn, axes=(0, 0))     # tangential coefficients
            for k, B in enumerate(reversed(Bb)):                # numpy axis k <-> tang[-1-k]
                dn = np.moveaxis(np.tensordot(B, dn, axes=(1, k)), 0, k)
            val = val + alpha * dn
        if beta != 0.0:
            g = np.full(val.shape, float(sd.get("g_const", 0.0)))
            if sd.get("g_table") is not None:
                g = g + np.asarray(sd["g_table"], dtype=np.float64).reshape(val.shape)
            val = val + beta * g
        rows = val
        for k, T in enumerate(reversed(Tb)):
            rows = np.moveaxis(np.tensordot(T, rows, axes=(1, k)), 0, k)
        full = np.multiply.outer(wa, rows)                      # normal axis first
        out += np.moveaxis(full, 0, dim - 1 - a)
    return out


def dirichlet_rows(pb: Problem, side_mask: int, rows: np.ndarray,
                   u: Optional[np.ndarray] = None) -> np.ndarray:
    """Row replacement for zero Dirichlet conditions (Section 4.3): the rows of the
    B-splines that do not vanish on a listed side (bit 2a: lower end of axis a, bit
    2a+1: upper end; B_0 and B_{N-1} of that axis under open knots) become identity
    rows, so rows[r] = u_r (operator applied to u), or 0 without u (right-hand side).
    Square systems only (rows indexed like the coefficients)."""
    out = np.array(rows, dtype=np.float64, copy=True)
    assert out.shape == pb.coef_shape()
    src = np.zeros_like(out) if u is None else np.asarray(u, dtype=np.float64)
    for a in range(pb.dim):
        ax = pb.dim - 1 - a
        for hi in (0, 1):
            if side_mask & (1 << (2 * a + hi)):
                idx = [slice(None)] * pb.dim
                idx[ax] = -1 if hi else 0
                out[tuple(idx)] = src[tuple(idx)]
    return out


# ---- refined test space (Section 2: more test elements than trial elements) ----------

def refined_cells(p: int, ne: int, rho: int) -> Tuple[np.ndarray, np.ndarray]:
    """Row i of the refined-test-space system sums the refined test B-splines
    Bhat_m, m in J_i = [a_i, b_i], of the open uniform knot vector with ne*rho elements:
    T_i = sum_{m in J_i} Bhat_m is 1 on the refined elements [a_i, b_i - p] (its cell)
    and ramps down over p refined elements on each side (none at the domain's ends).

    The cells partition the axis at the midpoints of consecutive Greville abscissae
    g_j = (t_{j+1} + ... + t_{j+p}) / p of the trial knots (element units), rounded to the
    nearest refined element boundary: cut_i = floor((rho (G_i + G_{i+1}) + p) / (2p)),
    G_j = p g_j, so that cell i sits at the centre of supp B_i (the reading of the
    paper's requirement that the N selected test functions be linearly independent)."""
    N = ne + p
    t = np.clip(np.arange(N + p + 1) - p, 0, ne)          # trial knots, element units
    G = np.array([int(t[j + 1:j + p + 1].sum()) for j in range(N)])
    cuts = [0] + [(rho * (int(G[i]) + int(G[i + 1])) + p) // (2 * p) for i in range(N - 1)] + [ne * rho]
    c = np.array(cuts, dtype=np.int64)
    return c[:-1].copy(), c[1:] - 1 + p


def _refined_axis(p: int, ne: int, rho: int, nq: int, lo: float, hi: float):
    """Sub-element Gauss points of one axis with the refined test functions and the
    trial basis (values and second derivatives) at each of them."""
    a, b = refined_cells(p, ne, rho)
    xi, w = gauss_legendre(nq)
    ns = ne * rho
    hs = (hi - lo) / ns
    k = np.repeat(np.arange(ns), nq)
    x = lo + hs * (k + (np.tile(xi, ns) + 1.0) / 2.0)
    W = np.tile(w, ns) * hs / 2.0
    N = ne + p
    T = np.zeros((N, len(x)))
    B = np.zeros((N, len(x)))
    B2 = np.zeros((N, len(x)))
    for q, xq in enumerate(x):
        bt = basis_eval(p, ns, xq, lo, hi, nder=0)[0]          # refined test basis
        tr = basis_eval(p, ne, xq, lo, hi, nder=2)             # trial basis
        csum = np.concatenate([[0.0], np.cumsum(bt)])
        T[:, q] = csum[b + 1] - csum[a]                        # sum of bt[a_i .. b_i]
        B[:, q] = tr[0]
        B2[:, q] = tr[2]
    return x, W, T, B, B2


def refined_matrix_1d(p: int, ne: int, rho: int, nq: int, kind: int, lo: float = 0.0,
                      hi: float = 1.0) -> np.ndarray:
    """M[i, j] = int T_i B_j (kind MAT_PG_MASS) or int T_i B_j'' (MAT_PG_LAP), with nq
    Gauss points on every refined element."""
    x, W, T, B, B2 = _refined_axis(p, ne, rho, nq, lo, hi)
    trial = B if kind == MAT_PG_MASS else B2
    return (T * W[None, :]) @ trial.T


def refined_rhs(pb: Problem, rho: Sequence[int], u: Optional[np.ndarray], alpha: float = 0.0,
                beta: float = 0.0, gamma: float = 0.0, sin_amp: float = 0.0) -> np.ndarray:
    """b_r = int T_r (alpha u_h + beta Lap u_h + gamma sin_amp prod_a sin(pi x_a)) with the
    tensor test functions T_r = prod_a T_{r_a}, evaluated at every point of the tensor
    sub-element Gauss grid."""
    dim = pb.dim
    ax = [_refined_axis(pb.p, pb.ne[a], int(rho[a]), pb.nq[a], pb.lo[a], pb.hi[a]) for a in range(dim)]

    def grid(mats):   # coefficient array (numpy order) -> values on the point grid
        v = np.asarray(u, dtype=np.float64)
        for k in range(dim):                                 # numpy axis k <-> mesh axis dim-1-k
            v = np.moveaxis(np.tensordot(mats[dim - 1 - k].T, v, axes=(1, k)), 0, k)
        return v

    shape = tuple(len(ax[a][0]) for a in reversed(range(dim)))
    f = np.zeros(shape)
    if u is not None and alpha != 0.0:
        f = f + alpha * grid([A[3] for A in ax])
    if u is not None and beta != 0.0:
        for t in range(dim):
            f = f + beta * grid([ax[a][4] if a == t else ax[a][3] for a in range(dim)])
    if gamma != 0.0 and sin_amp != 0.0:
        s = np.ones(())
        for a in reversed(range(dim)):
            s = np.multiply.outer(s, np.sin(np.pi * ax[a][0]))
        f = f + gamma * sin_amp * s
    for k in range(dim):
        a = dim - 1 - k
        TW = ax[a][2] * ax[a][1][None, :]
        f = np.moveaxis(np.tensordot(TW, f, axes=(1, k)), 0, k)
    return f


def refined_solve(pb: Problem, rho: Sequence[int], b: np.ndarray) -> np.ndarray:
    """Solves (P_z (x) P_y (x) P_x) x = b with the square refined-test-space mass
    matrices P_a = [int T_i B_j]: three families of 1D solves, x, then y, then z, each one
    call of numpy.linalg.solve (the alternating-directions solver of Section 4.1 with the
    Petrov-Galerkin matrices the refinement makes regular)."""
    x = np.array(b, dtype=np.float64, copy=True)
    for a in range(pb.dim):
        M = refined_matrix_1d(pb.p, pb.ne[a], int(rho[a]), pb.nq[a], MAT_PG_MASS, pb.lo[a], pb.hi[a])
        k = pb.dim - 1 - a
        lines = np.moveaxis(x, k, 0)
        sol = np.linalg.solve(M, lines.reshape(M.shape[0], -1))
        x = np.moveaxis(sol.reshape(lines.shape), 0, k)
    return np.ascontiguousarray(x)
