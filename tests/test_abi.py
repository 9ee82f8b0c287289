"""The C-ABI library (CPU, no device needed).

It loads, exports every function that include/ggem.h declares, the Python
binding wraps exactly those, and argument validation in ggem_plan_create /
ggem_solver_create rejects bad parameters before any device call.
"""
import ctypes
import os
import re

import pytest

import paper_1109_6587_amd.ggem as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ggem.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ggem_\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libggem.so not built")
    return B.load_library()


def test_header_parses():
    names = declared()
    assert "ggem_plan_create" in names and "ggem_fredholm_solve" in names
    assert len(names) >= 15


def test_every_declared_symbol_exported(lib):
    for name in declared():
        assert hasattr(lib, name), name
    assert sorted(B.EXPORTS) == declared()


def test_params_struct_matches_header():
    """The binding's Params mirrors the fields of ggem_params in order."""
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{(.*?)\} ggem_params;", txt, flags=re.S).group(1)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            names += [n.strip().lstrip("*") for n in decl.split(None, 1)[1].split(",")]
    names = [n.split()[-1] for n in names]
    assert names == [f for f, _ in B.Params._fields_]


def params(**kw):
    p = dict(Lx=8.0, Lz=8.0, H=2.0, alpha=3.0, rc=0.0, Nx=32, Nz=32, Ny=17, precision=B.FP64,
             sync_checks=1, max_src=10, max_tgt=10, cell_scale=0.0)
    p.update(kw)
    return B.Params(*[p[f] for f, _ in B.Params._fields_])


@pytest.mark.parametrize("bad,needle", [
    (dict(Lx=-1.0), "Lx"),
    (dict(H=0.0), "H must"),
    (dict(alpha=float("nan")), "alpha"),
    (dict(alpha=0.5), "half the period"),
    (dict(Nx=30 + 1), "Nx"),
    (dict(Nz=14 * 2 * 7), "Nx, Nz"),
    (dict(Ny=4), "Ny"),
    (dict(Ny=131), "Ny"),
    (dict(precision=7), "precision"),
    (dict(max_src=-1), "capacities"),
    (dict(cell_scale=4.5), "cell_scale"),
    (dict(cell_scale=-1.0), "cell_scale"),
    (dict(cell_scale=float("nan")), "cell_scale"),
])
def test_plan_create_rejects(lib, bad, needle):
    h = ctypes.c_void_p()
    rc = lib.ggem_plan_create(ctypes.byref(params(**bad)), None, ctypes.byref(h))
    assert rc == B.E_ARG
    assert not h.value
    assert needle in lib.ggem_last_error().decode()


def test_null_arguments(lib):
    assert lib.ggem_plan_create(None, None, None) == B.E_ARG
    assert lib.ggem_plan_destroy(None) == B.E_ARG
    assert lib.ggem_solver_destroy(None) == B.E_ARG
    out = ctypes.c_void_p()
    assert lib.ggem_solver_create(None, None, ctypes.byref(out)) == B.E_ARG
