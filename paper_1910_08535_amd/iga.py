"""Thin ctypes binding of the C ABI in include/iga.h (argument marshalling only).

Every computation runs in the HIP kernels of ``libiga.so``; torch is used only for
device memory and streams.  The binding refuses to run when the library is not
built -- there is no fallback path.

The raw functions carry the C names (``iga_create``, ``iga_rhs``, ...).  ``Mesh``
is a convenience wrapper that takes torch tensors (float64, CUDA, contiguous,
C-ordered (N_z, N_y, N_x), x fastest) and returns new tensors.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libiga.so")

IGA_OK, IGA_E_INVAL, IGA_E_UNSUPPORTED, IGA_E_NOMEM, IGA_E_DEVICE, IGA_E_AGAIN = 0, -1, -2, -3, -4, -5
IGA_E_SINGULAR = -6
SOLVE_NONE, SOLVE_LINES, SOLVE_PART_EXACT, SOLVE_PART_BLOCKDIAG = 0, 1, 2, 3
NOALLOC_MAX_DOUBLES = 1 << 23   # coefficients iga_explicit_step_noalloc takes at most
GALERKIN_BYPARTS, GALERKIN_LAPLACIAN, PG = 0, 1, 2
OP_MASS, OP_LAPLACE = 0, 1
SPANS_SUPPORT, SPANS_ELEMENT, SPANS_CUSTOM, SPANS_REFINED = 0, 1, 2, 3
TILE_2D_ROWS, TILE_3D_PLANES, TILE_3D_ROWS, TILE_2D_ORDER, TILE_3D_COLS, TILE_2D_STRIP = 1, 2, 4, 5, 6, 7
TILE_SOLVE_EXACT = 8   # partitioned solves: the reduced system always taken whole
TUNE_APPLY, TUNE_STEP, TUNE_MAX = 0, 1, 16
TILE_KEYS = {2: (TILE_2D_STRIP, TILE_2D_ROWS, TILE_2D_ORDER), 3: (TILE_3D_PLANES, TILE_3D_ROWS, TILE_3D_COLS)}
JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3

_P64 = C.POINTER(C.c_int64)


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("p", C.c_int32), ("ne", C.c_int64 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("nq", C.c_int32 * 3),
                ("spans", C.c_int32), ("nspan", C.c_int64 * 3),
                ("span_first", _P64 * 3), ("span_last", _P64 * 3), ("refine", C.c_int32 * 3)]


class Source(C.Structure):
    _fields_ = [("table", C.c_void_p), ("sin_amp", C.c_double)]


class Side(C.Structure):
    _fields_ = [("side", C.c_int32), ("g_table", C.c_void_p), ("g_const", C.c_double)]


class Job(C.Structure):
    _fields_ = [("p", C.c_int32), ("ne", C.c_int64 * 2), ("u", C.c_void_p),
                ("mass_out", C.c_void_p), ("lap_out", C.c_void_p)]


class Request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("p", C.c_int32), ("ne", C.c_int64 * 3),
                ("nsteps", C.c_int32), ("dt", C.c_double), ("sin_amp", C.c_double),
                ("u", C.c_void_p), ("mass_out", C.c_void_p), ("lap_out", C.c_void_p)]


REQ_RHS, REQ_STEP = 0, 1


class IGAError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_lib = None

# (name, argtypes)
_SIGS = {
    "iga_create": [C.POINTER(MeshDesc), C.c_void_p, C.POINTER(C.c_void_p)],
    "iga_destroy": [C.c_void_p],
    "iga_shape": [C.c_void_p, C.c_int32, C.c_int64 * 3, C.c_int64 * 3],
    "iga_assemble": [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p],
    "iga_rhs": [C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.c_double, C.c_double,
                C.POINTER(Source), C.c_void_p],
    "iga_apply": [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p],
    "iga_explicit_step": [C.c_void_p, C.c_void_p, C.c_double, C.POINTER(Source), C.c_int32],
    "iga_explicit_step_noalloc": [C.c_void_p, C.c_void_p, C.c_double, C.POINTER(Source), C.c_int32],
    "iga_solve": [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p],
    "iga_solve_info": [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
    "iga_boundary_terms": [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(Side), C.c_void_p, C.c_double,
                           C.c_double, C.c_void_p],
    "iga_dirichlet_rows": [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p],
    "iga_galerkin_step": [C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.POINTER(Source),
                          C.c_int32],
    "iga_strerror": [C.c_int],
    "iga_copy_probe": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p],
    "iga_set_tile": [C.c_void_p, C.c_int32, C.c_int32],
    "iga_get_tile": [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)],
    "iga_autotune": [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.POINTER(C.c_int32)],
    "iga_batch_create": [C.c_void_p, C.c_size_t, C.c_int32, C.POINTER(C.c_void_p)],
    "iga_batch_submit": [C.c_void_p, C.POINTER(Job), C.c_int32, C.POINTER(C.c_uint64)],
    "iga_batch_flush": [C.c_void_p],
    "iga_batch_poll": [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32)],
    "iga_batch_wait": [C.c_void_p],
    "iga_batch_autotune": [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_float)],
    "iga_batch_destroy": [C.c_void_p],
    "iga_server_create": [C.c_int32, C.c_size_t, C.c_size_t, C.POINTER(C.c_void_p)],
    "iga_server_submit": [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
    "iga_server_progress": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                            C.POINTER(C.c_int32)],
    "iga_server_stats": [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t),
                         C.POINTER(C.c_int64), C.POINTER(C.c_double)],
    "iga_server_cache_stats": [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_int64)],
    "iga_server_destroy": [C.c_void_p],
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.argtypes = args
            fn.restype = C.c_char_p if name == "iga_strerror" else C.c_int
        _lib = L
    return _lib


def exported_symbols() -> list:
    L = lib()
    return [n for n in _SIGS if hasattr(L, n)]


def strerror(code: int) -> str:
    try:
        return lib().iga_strerror(code).decode()
    except Exception:  # library missing: still report the number
        return f"error {code}"


def _check(rc: int, where: str) -> None:
    if rc != IGA_OK:
        raise IGAError(rc, where)


# ---- raw C calls (same names as the C ABI) -------------------------------------

def iga_create(desc: MeshDesc, stream: int) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().iga_create(C.byref(desc), C.c_void_p(stream), C.byref(h)), "iga_create")
    return h


def iga_destroy(h) -> None:
    _check(lib().iga_destroy(h), "iga_destroy")


def iga_shape(h, form: int) -> Tuple[Tuple[int, ...], Tuple[int, ...]]:
    rows, cols = (C.c_int64 * 3)(), (C.c_int64 * 3)()
    _check(lib().iga_shape(h, form, rows, cols), "iga_shape")
    return tuple(rows), tuple(cols)


def iga_assemble(h, form: int, op: int, bands_ptr: int) -> None:
    _check(lib().iga_assemble(h, form, op, C.c_void_p(bands_ptr)), "iga_assemble")


def iga_rhs(h, form: int, u_ptr: Optional[int], alpha: float, beta: float, gamma: float,
            src: Optional[Source], b_ptr: int) -> None:
    _check(lib().iga_rhs(h, form, C.c_void_p(u_ptr) if u_ptr else None, alpha, beta, gamma,
                         C.byref(src) if src is not None else None, C.c_void_p(b_ptr)),
           "iga_rhs")


def iga_apply(h, form: int, u_ptr: int, mass_ptr: Optional[int], lap_ptr: Optional[int]) -> None:
    _check(lib().iga_apply(h, form, C.c_void_p(u_ptr), C.c_void_p(mass_ptr) if mass_ptr else None,
                           C.c_void_p(lap_ptr) if lap_ptr else None), "iga_apply")


def iga_explicit_step(h, u_ptr: int, dt: float, src: Optional[Source], nsteps: int) -> None:
    _check(lib().iga_explicit_step(h, C.c_void_p(u_ptr), dt,
                                   C.byref(src) if src is not None else None, nsteps),
           "iga_explicit_step")


def iga_explicit_step_noalloc(h, u_ptr: int, dt: float, src: Optional[Source], nsteps: int) -> None:
    _check(lib().iga_explicit_step_noalloc(h, C.c_void_p(u_ptr), dt,
                                           C.byref(src) if src is not None else None, nsteps),
           "iga_explicit_step_noalloc")


def iga_boundary_terms(h, form: int, sides, u_ptr: int, alpha: float, beta: float, b_ptr: int) -> None:
    arr = (Side * max(1, len(sides)))(*sides)
    _check(lib().iga_boundary_terms(h, form, len(sides), arr, C.c_void_p(u_ptr), alpha, beta,
                                    C.c_void_p(b_ptr)), "iga_boundary_terms")


def iga_dirichlet_rows(h, form: int, side_mask: int, u_ptr: int, rows_ptr: int) -> None:
    _check(lib().iga_dirichlet_rows(h, form, side_mask, C.c_void_p(u_ptr), C.c_void_p(rows_ptr)),
           "iga_dirichlet_rows")


def iga_solve(h, form: int, b_ptr: int, x_ptr: int) -> None:
    _check(lib().iga_solve(h, form, C.c_void_p(b_ptr), C.c_void_p(x_ptr)), "iga_solve")


def iga_solve_info(h, axis: int) -> Tuple[int, int]:
    scheme, chunks = C.c_int32(), C.c_int32()
    _check(lib().iga_solve_info(h, axis, C.byref(scheme), C.byref(chunks)), "iga_solve_info")
    return scheme.value, chunks.value


def iga_galerkin_step(h, form: int, u_ptr: int, dt: float, src: Optional[Source],
                      nsteps: int) -> None:
    _check(lib().iga_galerkin_step(h, form, C.c_void_p(u_ptr), dt,
                                   C.byref(src) if src is not None else None, nsteps),
           "iga_galerkin_step")


def iga_set_tile(h, key: int, value: int) -> None:
    _check(lib().iga_set_tile(h, key, value), "iga_set_tile")


def iga_autotune(h, op: int, reps: int):
    """Times the candidate tiles (the list of include/iga.h); returns their microseconds."""
    import numpy as np
    times = np.zeros(TUNE_MAX, dtype=np.float32)
    n = C.c_int32(0)
    _check(lib().iga_autotune(h, op, reps, times.ctypes.data, C.byref(n)), "iga_autotune")
    return times[: n.value].copy()


def iga_get_tile(h, key: int) -> int:
    v = C.c_int32()
    _check(lib().iga_get_tile(h, key, C.byref(v)), "iga_get_tile")
    return v.value


def iga_copy_probe(src_ptr: int, a_ptr: int, b_ptr: int, n: int, stream: int) -> None:
    _check(lib().iga_copy_probe(C.c_void_p(src_ptr), C.c_void_p(a_ptr), C.c_void_p(b_ptr), n,
                                C.c_void_p(stream)), "iga_copy_probe")


# ---- torch convenience layer ----------------------------------------------------

def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int:
    import torch
    if t is None:
        return 0
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return int(t.data_ptr())


class Mesh:
    """One context: a tensor-product B-spline space with its Gauss rule and spans.

    ne, nq, lo, hi are per axis in (x, y, z) order.  ``spans`` is "support",
    "element", "refined" (with ``refine``: refined elements per trial element, per
    axis) or a list of per-axis (first, last) integer arrays (custom)."""

    def __init__(self, dim: int, p: int, ne: Sequence[int], nq: Sequence[int],
                 lo: Optional[Sequence[float]] = None, hi: Optional[Sequence[float]] = None,
                 spans="support", stream=None, refine: Optional[Sequence[int]] = None):
        import numpy as np
        self.stream = stream
        d = MeshDesc()
        d.dim, d.p = dim, p
        lo = list(lo) if lo is not None else [0.0] * dim
        hi = list(hi) if hi is not None else [1.0] * dim
        self._keep = []
        for a in range(3):
            real = a < dim
            d.ne[a] = int(ne[a]) if real else 1
            d.nq[a] = int(nq[a]) if real else 1
            d.lo[a] = float(lo[a]) if real else 0.0
            d.hi[a] = float(hi[a]) if real else 1.0
        if isinstance(spans, str):
            d.spans = {"support": SPANS_SUPPORT, "element": SPANS_ELEMENT, "refined": SPANS_REFINED}[spans]
            if spans == "refined":
                for a in range(dim):
                    d.refine[a] = int(refine[a])
        else:
            d.spans = SPANS_CUSTOM
            for a in range(dim):
                f = np.ascontiguousarray(spans[a][0], dtype=np.int64)
                l = np.ascontiguousarray(spans[a][1], dtype=np.int64)
                self._keep += [f, l]
                d.nspan[a] = len(f)
                d.span_first[a] = f.ctypes.data_as(_P64)
                d.span_last[a] = l.ctypes.data_as(_P64)
        self.dim, self.p = dim, p
        self.ne = tuple(int(v) for v in ne[:dim])
        self.nq = tuple(int(v) for v in nq[:dim])
        self.h = iga_create(d, _stream_handle(stream))
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            iga_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tile(self, key: int, value: int) -> None:
        iga_set_tile(self.h, key, value)

    def get_tile(self, key: int) -> int:
        return iga_get_tile(self.h, key)

    def tile(self) -> dict:
        """The context's tile setting (the keys its dimension uses)."""
        names = {TILE_2D_STRIP: "strip", TILE_2D_ROWS: "rows", TILE_2D_ORDER: "order",
                 TILE_3D_PLANES: "planes", TILE_3D_ROWS: "rows", TILE_3D_COLS: "cols"}
        return {names[k]: self.get_tile(k) for k in TILE_KEYS.get(self.dim, ())}

    def autotune(self, op: int = TUNE_APPLY, reps: int = 20):
        """Picks the fastest candidate tile for op (TUNE_APPLY or TUNE_STEP) and keeps it for
        this context and later ones of the same size class; returns the candidates'
        microseconds per launch."""
        return iga_autotune(self.h, op, reps)

    def shape(self, form: int) -> Tuple[int, ...]:
        rows, _ = iga_shape(self.h, form)
        return tuple(reversed(rows[: self.dim]))

    def coef_shape(self) -> Tuple[int, ...]:
        _, cols = iga_shape(self.h, PG)
        return tuple(reversed(cols[: self.dim]))

    def _new(self, shape):
        import torch
        return torch.empty(shape, dtype=torch.float64, device="cuda")

    def _src(self, f_table, sin_amp) -> Optional[Source]:
        if f_table is None and sin_amp == 0.0:
            return None
        s = Source()
        s.table = C.c_void_p(_ptr(f_table)) if f_table is not None else None
        s.sin_amp = float(sin_amp)
        return s

    def rhs(self, form: int, u=None, alpha: float = 0.0, beta: float = 0.0, gamma: float = 0.0,
            f_table=None, sin_amp: float = 0.0, out=None):
        b = out if out is not None else self._new(self.shape(form))
        iga_rhs(self.h, form, _ptr(u) if u is not None else 0, alpha, beta, gamma,
                self._src(f_table, sin_amp), _ptr(b))
        return b

    def apply(self, form: int, u, mass: bool = True, lap: bool = True, out_mass=None, out_lap=None):
        m = out_mass if out_mass is not None else (self._new(self.shape(form)) if mass else None)
        l = out_lap if out_lap is not None else (self._new(self.shape(form)) if lap else None)
        iga_apply(self.h, form, _ptr(u), _ptr(m) if m is not None else 0,
                  _ptr(l) if l is not None else 0)
        return m, l

    def explicit_step(self, u, dt: float, f_table=None, sin_amp: float = 0.0, nsteps: int = 1):
        """In place on u (returned)."""
        iga_explicit_step(self.h, _ptr(u), dt, self._src(f_table, sin_amp), nsteps)
        return u

    def solve(self, b, form: int = GALERKIN_LAPLACIAN, out=None):
        """x = (M_z (x) M_y (x) M_x)^{-1} b with the Galerkin mass; out may be b."""
        x = out if out is not None else self._new(self.coef_shape())
        iga_solve(self.h, form, _ptr(b), _ptr(x))
        return x

    def solve_info(self, axis: int) -> Tuple[int, int]:
        """(scheme, chunks per line) of the solves along an axis (SOLVE_* constants)."""
        return iga_solve_info(self.h, axis)

    def galerkin_step(self, u, dt: float, form: int = GALERKIN_LAPLACIAN, f_table=None,
                      sin_amp: float = 0.0, nsteps: int = 1):
        """Consistent-mass Euler steps in place on u (returned)."""
        iga_galerkin_step(self.h, form, _ptr(u), dt, self._src(f_table, sin_amp), nsteps)
        return u

    def boundary_terms(self, form: int, sides, b, u=None, alpha: float = 0.0, beta: float = 0.0):
        """b += sum over sides of int_side T_r (alpha du_h/dn + beta G); sides: list of
        (side, g_table or None, g_const).  Returns b."""
        recs = []
        for sd, tab, c in sides:
            recs.append(Side(int(sd), C.c_void_p(_ptr(tab)) if tab is not None else None, float(c)))
        iga_boundary_terms(self.h, form, recs, _ptr(u) if u is not None else 0, alpha, beta, _ptr(b))
        return b

    def dirichlet_rows(self, form: int, side_mask: int, rows, u=None):
        """Identity rows on the listed sides (rows[r] = u[r], or 0 without u).  Returns rows."""
        iga_dirichlet_rows(self.h, form, side_mask, _ptr(u) if u is not None else 0, _ptr(rows))
        return rows

    def assemble(self, form: int, op: int = OP_LAPLACE):
        """Banded factors, tensor of shape (dim, 2, Rmax, 2p+1)."""
        import torch
        rows, _ = iga_shape(self.h, form)
        rmax = max(rows[: self.dim])
        bands = torch.zeros((self.dim, 2, rmax, 2 * self.p + 1), dtype=torch.float64, device="cuda")
        iga_assemble(self.h, form, op, _ptr(bands))
        return bands


def bands_to_dense(band, nrows: int, ncols: int, p: int):
    """Host helper: one banded factor (Rmax, 2p+1) -> dense (nrows, ncols) numpy array."""
    import numpy as np
    band = np.asarray(band)
    out = np.zeros((nrows, ncols))
    for r in range(nrows):
        for k in range(2 * p + 1):
            c = r + k - p
            if 0 <= c < ncols:
                out[r, c] = band[r, k]
    return out


# ---- batches ----------------------------------------------------------------------

class Batch:
    """Many independent 2D fused PG applies in one persistent launch (iga_batch_*).

    Tensors passed to submit() must stay alive until their job is done."""

    def __init__(self, mem_budget_bytes: int = 0, max_jobs: int = 1024, stream=None):
        self.stream = stream
        self.h = C.c_void_p()
        _check(lib().iga_batch_create(C.c_void_p(_stream_handle(stream)), mem_budget_bytes,
                                      max_jobs, C.byref(self.h)), "iga_batch_create")

    def submit(self, jobs: Sequence[Tuple[int, Tuple[int, int], object, object, object]]) -> list:
        """jobs: (p, (nx, ny), u, mass_out, lap_out) with torch tensors; returns tickets."""
        arr = (Job * len(jobs))()
        for k, (p, ne, u, m, l) in enumerate(jobs):
            arr[k].p = p
            arr[k].ne[0], arr[k].ne[1] = ne
            arr[k].u, arr[k].mass_out, arr[k].lap_out = _ptr(u), _ptr(m), _ptr(l)
        tickets = (C.c_uint64 * max(1, len(jobs)))()
        _check(lib().iga_batch_submit(self.h, arr, len(jobs), tickets), "iga_batch_submit")
        return list(tickets)[: len(jobs)]

    def try_submit(self, jobs) -> Optional[list]:
        """Like submit(), but returns None when the batch answers IGA_E_AGAIN."""
        try:
            return self.submit(jobs)
        except IGAError as e:
            if e.code == IGA_E_AGAIN:
                return None
            raise

    def flush(self) -> None:
        _check(lib().iga_batch_flush(self.h), "iga_batch_flush")

    def poll(self, ticket: int) -> int:
        st = C.c_int32()
        _check(lib().iga_batch_poll(self.h, ticket, C.byref(st)), "iga_batch_poll")
        return st.value

    def wait(self) -> None:
        _check(lib().iga_batch_wait(self.h), "iga_batch_wait")

    def autotune(self, reps: int = 3) -> Tuple[int, float]:
        """(best chunk rows, milliseconds per launch of the queued jobs with it)."""
        best = C.c_int32()
        ms = C.c_float()
        _check(lib().iga_batch_autotune(self.h, reps, C.byref(best), C.byref(ms)),
               "iga_batch_autotune")
        return best.value, ms.value

    def close(self) -> None:
        if getattr(self, "h", None):
            _check(lib().iga_batch_destroy(self.h), "iga_batch_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- serving ----------------------------------------------------------------------

def request_dtype():
    """numpy record layout of iga_request (checked against the ctypes structure)."""
    import numpy as np
    dt = np.dtype({"names": [f[0] for f in Request._fields_],
                   "formats": [np.int32, np.int32, np.int32, (np.int64, 3), np.int32, np.float64,
                               np.float64, np.uint64, np.uint64, np.uint64],
                   "offsets": [getattr(Request, f[0]).offset for f in Request._fields_],
                   "itemsize": C.sizeof(Request)})
    return dt


class NativeServer:
    """The library's request loop (iga_server_*).  Buffers of submitted requests must stay
    alive until they are reported done."""

    def __init__(self, nstreams: int = 4, budget_bytes: int = 200 * 10**9,
                 cache_bytes: int = 16 << 30):
        import numpy as np
        self.h = C.c_void_p()
        _check(lib().iga_server_create(nstreams, budget_bytes, cache_bytes, C.byref(self.h)),
               "iga_server_create")
        self.dtype = request_dtype()
        self._cap = 4096
        self._done = np.zeros(self._cap, dtype=np.uint64)
        self._time = np.zeros(self._cap, dtype=np.float64)
        self._state = np.zeros(self._cap, dtype=np.int32)
        self._launch = np.zeros(self._cap, dtype=np.int64)

    def submit(self, recs) -> "object":
        """recs: numpy array of request_dtype(); returns the tickets (numpy uint64)."""
        import numpy as np
        recs = np.ascontiguousarray(recs, dtype=self.dtype)
        tickets = np.zeros(max(1, len(recs)), dtype=np.uint64)
        _check(lib().iga_server_submit(self.h, recs.ctypes.data, len(recs), tickets.ctypes.data),
               "iga_server_submit")
        return tickets[: len(recs)]

    def progress(self):
        """Completions observed now: (tickets, times, states, batch launch indices)."""
        n = C.c_int32()
        _check(lib().iga_server_progress(self.h, self._done.ctypes.data, self._time.ctypes.data,
                                         self._state.ctypes.data, self._launch.ctypes.data,
                                         self._cap, C.byref(n)), "iga_server_progress")
        k = n.value
        return (self._done[:k].copy(), self._time[:k].copy(), self._state[:k].copy(),
                self._launch[:k].copy())

    def stats(self):
        used, peak, launches, now = C.c_size_t(), C.c_size_t(), C.c_int64(), C.c_double()
        _check(lib().iga_server_stats(self.h, C.byref(used), C.byref(peak), C.byref(launches),
                                      C.byref(now)), "iga_server_stats")
        return used.value, peak.value, launches.value, now.value

    def cache_stats(self):
        """(device bytes of the cached contexts, their number)."""
        b, n = C.c_size_t(), C.c_int64()
        _check(lib().iga_server_cache_stats(self.h, C.byref(b), C.byref(n)), "iga_server_cache_stats")
        return b.value, n.value

    def close(self) -> None:
        if getattr(self, "h", None):
            _check(lib().iga_server_destroy(self.h), "iga_server_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
