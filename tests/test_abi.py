"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/pst.h declares, and host-side validation rejects bad
arguments before any device call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pst.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pst_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def pst():
    from paper_1808_01309_amd import pst as m
    return m


def test_header_declares_functions():
    names = declared_functions()
    assert "pst_plan_create" in names and "pst_step" in names and len(names) >= 15


def test_every_declared_symbol_is_exported(pst):
    lib = ctypes.CDLL(pst.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(declared_functions()) == sorted(pst.EXPORTED)


def test_status_strings(pst):
    assert pst.lib.pst_status_str(0) == b"ok"
    assert pst.lib.pst_status_str(2) == b"unsupported grid size"
    assert pst.lib.pst_status_str(99) == b"unknown status"


@pytest.mark.parametrize("n,ok", [(16, 1), (24, 1), (512, 1), (1024, 1), (0, 0), (7, 0), (40, 0), (2048, 0)])
def test_supported_n(pst, n, ok):
    assert pst.lib.pst_supported_n(n) == ok


def _create(pst, **kw):
    base = dict(n=32, solver=0, precision=0, rk_order=4, nu=0.01, eta=0.01, dt=1e-3, dealias=0, flags=0)
    base.update(kw)
    p = pst.pst_params(**base)
    h = ctypes.c_void_p()
    s = pst.lib.pst_plan_create(ctypes.byref(p), None, ctypes.byref(h))
    return s, h


@pytest.mark.parametrize("kw,status", [
    (dict(n=7), 2), (dict(n=0), 2), (dict(n=40), 2),
    (dict(solver=5), 1), (dict(precision=3), 1), (dict(rk_order=3), 1),
    (dict(dt=0.0), 1), (dict(dt=-1.0), 1), (dict(nu=-1.0), 1), (dict(nu=float("nan")), 1),
    (dict(solver=1, eta=-2.0), 1), (dict(solver=2, eta=-1.0), 1), (dict(solver=2, nbv=float("inf")), 1),
    (dict(dealias=3), 6), (dict(flags=0x100), 1),
    (dict(nx=40), 2), (dict(nz=7), 2), (dict(ny=-2), 1), (dict(lx=-1.0), 1), (dict(lz=float("nan")), 1),
    (dict(ny=16, dealias=1), 6), (dict(ly=3.0, dealias=1), 6), (dict(solver=3, dealias=1), 6),
    (dict(solver=3, alpha=float("inf")), 1),
])
def test_plan_create_rejects_bad_params(pst, kw, status):
    s, h = _create(pst, **kw)
    assert s == status
    assert not h.value
    assert len(pst.lib.pst_last_error(None)) > 0


def test_null_arguments(pst):
    assert pst.lib.pst_plan_create(None, None, None) == 1
    p = pst.pst_params(n=32, solver=0, precision=0, rk_order=4, nu=0.0, eta=0.0, dt=1e-3, dealias=0, flags=0)
    assert pst.lib.pst_plan_create(ctypes.byref(p), None, None) == 1
    pst.lib.pst_plan_destroy(None)  # no-op
    assert pst.lib.pst_step(None, 1) == 1
    assert pst.lib.pst_energy(None, None) == 1
    assert pst.lib.pst_query(None, None) == 1
