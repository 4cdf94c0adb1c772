"""hl_norms_noalloc: the norms with their block partials in the library's
file-scope device array instead of the plan's buffer (for callers that
cannot allocate).  Called through the C ABI twice in a row, the second time
on a smaller plan, and checked against hl_norms (the same kernels and the
same fixed summation order, so the sums agree to rounding of the final
additions: relative 1e-13), in FP64, FP32 and FP32_COMP, periodic and walled
plans, up to the largest plane count its scratch holds (3D m = 3)."""

import ctypes
import sys

import numpy as np
import pytest

from paper_1808_10481_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1808_10481_amd import hl  # noqa: E402


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _noalloc(plan, p, u):
    out = (ctypes.c_double * 2)()
    hl._check(hl.lib().hl_norms_noalloc(plan._h, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                        out))
    return np.array([out[0], out[1]])


def _plan_state(d, m, K, prec, boundary, seed):
    plan = hl.Plan(d, m, K, cfl=0.5, precision=prec, boundary=boundary)
    rng = np.random.default_rng(seed)
    ps, us = plan.host_shapes()
    P0 = inputs.random_data(rng, d, m, ps[:d])
    if boundary == "walls":
        P0 = inputs.zero_on_walls(P0, d)
    p, u = plan.alloc()
    plan.init(p, u, P0, rng.uniform(-1, 1, us))
    return plan, p, u


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_comp"])
@pytest.mark.parametrize("first,second", [
    ((3, 3, (20, 12, 9), "periodic"), (2, 2, (17, 5), "periodic")),
    ((2, 5, (40, 33), "walls"), (1, 1, (7,), "periodic")),
    ((3, 2, (24, 16, 8), "walls"), (3, 1, (5, 4, 3), "walls")),
])
def test_noalloc_norms_match_hl_norms_twice(prec, first, second):
    for k, (d, m, K, boundary) in enumerate((first, second)):
        _say(f"[noalloc] call {k + 1}: d={d} m={m} K={K} {prec} {boundary}")
        plan, p, u = _plan_state(d, m, K, prec, boundary, 10 + k)
        ref = np.array(plan.norms(p, u))
        got = _noalloc(plan, p, u)
        assert np.allclose(got, ref, rtol=1e-13, atol=0), (got, ref)
        plan.close()


def test_noalloc_rejects_null_and_reports_nonfinite():
    plan, p, u = _plan_state(2, 1, (8, 8), "fp64", "periodic", 3)
    out = (ctypes.c_double * 2)()
    st = hl.lib().hl_norms_noalloc(plan._h, None, ctypes.c_void_p(u.data_ptr()), out)
    assert st == hl.HL_ERR_ARG
    p[5] = float("nan")
    st = hl.lib().hl_norms_noalloc(plan._h, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(u.data_ptr()), out)
    assert st == hl.HL_ERR_NONFINITE
    plan.close()
