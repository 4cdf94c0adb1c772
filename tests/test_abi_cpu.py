"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/hl.h declares, and rejects bad problems on the host before any
device call."""

import ctypes
import os
import re

import pytest

from paper_1808_10481_amd import hl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hl.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:hl_status|const char\*)\s+(hl_\w+)\s*\(", txt, re.M)))


def test_header_declarations_match_binding():
    assert _declared() == sorted(hl.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = hl.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def _plan_status(**kw):
    pr = hl.make_problem(**kw)
    h = ctypes.c_void_p()
    st = hl.lib().hl_plan(ctypes.byref(pr), ctypes.byref(h))
    return st, hl.lib().hl_last_error().decode(), h


@pytest.mark.parametrize("kw,want", [
    (dict(d=0, m=1, cells=(8,)), hl.HL_ERR_ARG),
    (dict(d=4, m=1, cells=(8,)), hl.HL_ERR_ARG),
    (dict(d=1, m=-1, cells=(8,)), hl.HL_ERR_ARG),
    (dict(d=1, m=8, cells=(8,)), hl.HL_ERR_UNSUPPORTED),
    (dict(d=2, m=6, cells=(8, 8)), hl.HL_ERR_UNSUPPORTED),
    (dict(d=3, m=4, cells=(8, 8, 8)), hl.HL_ERR_UNSUPPORTED),
    (dict(d=1, m=1, cells=(1,)), hl.HL_ERR_ARG),
    (dict(d=2, m=1, cells=(8, 1)), hl.HL_ERR_ARG),
    (dict(d=1, m=1, cells=(8,), c=0.0), hl.HL_ERR_ARG),
    (dict(d=1, m=1, cells=(8,), c=float("nan")), hl.HL_ERR_ARG),
    (dict(d=1, m=1, cells=(8,), length=(-1.0,)), hl.HL_ERR_ARG),
    (dict(d=1, m=1, cells=(8,), dt=-1.0), hl.HL_ERR_ARG),
    (dict(d=1, m=1, cells=(8,), dt=0.0, cfl=1.0), hl.HL_ERR_CFL),
    (dict(d=1, m=1, cells=(8,), dt=0.0, cfl=0.0), hl.HL_ERR_CFL),
    (dict(d=1, m=1, cells=(8,), dt=0.125), hl.HL_ERR_CFL),        # c dt / h = 1
    (dict(d=2, m=1, cells=(8, 16), length=(1.0, 1.0), dt=0.07), hl.HL_ERR_CFL),  # min h = 1/16
])
def test_plan_rejects_bad_problems(kw, want):
    st, msg, h = _plan_status(**kw)
    assert st == want, (st, msg)
    assert msg
    assert not h.value


def test_plan_rejects_unknown_precision_and_oversized_planes():
    st, msg, h = _plan_status(d=1, m=1, cells=(8,), precision="fp64")
    pr = hl.make_problem(1, 1, (8,))
    pr.precision = 3
    h = ctypes.c_void_p()
    assert hl.lib().hl_plan(ctypes.byref(pr), ctypes.byref(h)) == hl.HL_ERR_ARG
    # one FP32 (or FP32_COMP hi) plane of 2^30 nodes is 4 GiB: refused before any device call
    for prec in ("fp32", "fp32_comp"):
        st, msg, h = _plan_status(d=3, m=0, cells=(1024, 1024, 1024), precision=prec)
        assert st == hl.HL_ERR_UNSUPPORTED and "4 GiB" in msg, (prec, st, msg)
    st, msg, h = _plan_status(d=3, m=0, cells=(1024, 1024, 512), precision="fp64")
    assert st == hl.HL_ERR_UNSUPPORTED and "4 GiB" in msg
    # walls: the ghost-padded velocity array sets the size (1023 x 1023 x 1022 cells pad to 1025 x 1025 x 1024 >= 2^30 nodes)
    st, msg, h = _plan_status(d=3, m=0, cells=(1023, 1023, 1022), precision="fp32", boundary="walls")
    assert st == hl.HL_ERR_UNSUPPORTED and "4 GiB" in msg


def test_plan_rejects_null_and_reserved():
    h = ctypes.c_void_p()
    assert hl.lib().hl_plan(None, ctypes.byref(h)) == hl.HL_ERR_ARG
    pr = hl.make_problem(1, 1, (8,))
    pr.reserved[1] = 1
    assert hl.lib().hl_plan(ctypes.byref(pr), ctypes.byref(h)) == hl.HL_ERR_ARG
    pr = hl.make_problem(1, 1, (8,))
    pr.boundary = 2
    assert hl.lib().hl_plan(ctypes.byref(pr), ctypes.byref(h)) == hl.HL_ERR_ARG


def test_adjoint_rejects_null_plan():
    st = hl.lib().hl_adjoint_step(None, None, None, None, None, None, 1, None)
    assert st == hl.HL_ERR_ARG
    assert hl.lib().hl_adjoint_step_var(None, None, None, None, None, None) == hl.HL_ERR_ARG
    assert hl.lib().hl_kappa_grad(None, None, None, 0) == hl.HL_ERR_ARG


def test_null_plan_arguments():
    assert hl.lib().hl_plan_destroy(None) == hl.HL_OK
    assert hl.lib().hl_step(None, None, None, 1, None) == hl.HL_ERR_ARG
    assert hl.lib().hl_plan_info(None, None) == hl.HL_ERR_ARG
