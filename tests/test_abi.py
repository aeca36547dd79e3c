"""The C-ABI library loads and exports every entry point that include/iga.h declares,
and rejects bad descriptors before touching the device (CPU only)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "iga.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(iga_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def iga():
    from paper_1910_08535_amd import iga as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1910_08535_amd import build
        build.build()
    return m


def test_every_declared_symbol_is_exported(iga):
    names = _declared()
    assert "iga_create" in names and "iga_batch_submit" in names and len(names) >= 14
    L = C.CDLL(iga.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_strerror(iga):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert iga.strerror(code) and "unknown" not in iga.strerror(code)
    assert "unknown" in iga.strerror(-99)


def _desc(iga, **kw):
    d = iga.MeshDesc()
    d.dim, d.p = kw.get("dim", 2), kw.get("p", 2)
    for a in range(3):
        d.ne[a] = kw.get("ne", (8, 8, 8))[a]
        d.nq[a] = kw.get("nq", (3, 3, 3))[a]
        d.lo[a], d.hi[a] = 0.0, kw.get("hi", 1.0)
    d.spans = kw.get("spans", 0)
    for a in range(3):
        d.refine[a] = kw.get("refine", (4, 4, 4))[a]
    return d


@pytest.mark.parametrize("kw,code", [
    (dict(dim=0), -2), (dict(dim=4), -2), (dict(p=1), -2), (dict(p=4), -2),
    (dict(nq=(0, 3, 3)), -2), (dict(nq=(3, 17, 3)), -2),
    (dict(ne=(0, 8, 8)), -1), (dict(hi=0.0), -1), (dict(spans=7), -1),
    (dict(ne=(50000, 50000, 8)), -1),
    # 2D arrays and band tables must stay below 4 GiB (32-bit buffer offsets)
    (dict(ne=(23171, 23171, 1)), -1), (dict(p=3, ne=(76_700_000, 2, 1)), -1),
    # refined test space: refinement 1..64, cells non-empty, rows inside the band
    (dict(spans=3, refine=(0, 4, 4)), -1), (dict(spans=3, refine=(4, 65, 4)), -1),
    (dict(spans=3, refine=(1, 4, 4)), -1), (dict(spans=3, refine=(2, 4, 4)), -1),
    (dict(spans=3, p=3, refine=(4, 3, 4)), -1), (dict(spans=4), -1),
])
def test_create_rejects_bad_descriptors(iga, kw, code):
    h = C.c_void_p()
    assert iga.lib().iga_create(C.byref(_desc(iga, **kw)), None, C.byref(h)) == code
    assert not h.value


def test_custom_span_outside_support_rejected(iga):
    import numpy as np
    d = _desc(iga, dim=1, ne=(4, 1, 1), spans=2)
    first = np.array([0, 0, 1, 2, 3, 3], dtype=np.int64)
    last = np.array([0, 1, 3, 2, 3, 3], dtype=np.int64)   # row 2: [1,3] leaves supp B_2 = [0,2]
    d.nspan[0] = 6
    d.span_first[0] = first.ctypes.data_as(C.POINTER(C.c_int64))
    d.span_last[0] = last.ctypes.data_as(C.POINTER(C.c_int64))
    h = C.c_void_p()
    assert iga.lib().iga_create(C.byref(d), None, C.byref(h)) == -1


def test_null_arguments(iga):
    L = iga.lib()
    assert L.iga_create(None, None, None) == -1
    assert L.iga_destroy(None) == -1
    assert L.iga_rhs(None, 2, None, 1.0, 0.0, 0.0, None, None) == -1
    assert L.iga_apply(None, 2, None, None, None) == -1
    assert L.iga_explicit_step(None, None, 0.1, None, 1) == -1
    assert L.iga_solve(None, 1, None, None) == -1
    assert L.iga_galerkin_step(None, 1, None, 0.1, None, 1) == -1
    assert L.iga_boundary_terms(None, 2, 0, None, None, 0.0, 0.0, None) == -1
    assert L.iga_dirichlet_rows(None, 2, 1, None, None) == -1
