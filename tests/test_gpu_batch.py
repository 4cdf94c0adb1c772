"""Batched shots (hl_batch_*): uneven grids, time steps, coefficients and
precisions per batch, advanced with one launch per half-step, must equal each
plan's own hl_step bit for bit (the same kernels and arithmetic run)."""

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


def _shots(d, m, prec, sizes, rng, var=False):
    plans, states = [], []
    for K in sizes:
        c = float(rng.uniform(0.8, 1.8))
        plan = hl.Plan(d, m, K, cfl=float(rng.uniform(0.3, 0.9)), c=c, precision=prec)
        if var:
            amps = tuple(rng.uniform(0.05, 0.2, d))
            waves = tuple(int(w) for w in rng.integers(1, 3, d))
            plan.set_kappa(inputs.kappa_sines(d, m, K, (1.0,) * d, amps, waves, "primal"),
                           inputs.kappa_sines(d, m, K, (1.0,) * d, amps, waves, "dual"))
        p, u = plan.alloc()
        plan.init(p, u, inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d))
        plans.append(plan)
        states.append((p, u))
    return plans, states


@pytest.mark.parametrize("d,m,prec,sizes,var", [
    (2, 3, "fp32", [(64, 48), (100, 37), (33, 80), (128, 128), (2, 3)], False),
    (2, 2, "fp64", [(40, 24), (17, 9), (64, 64)], True),
    (1, 5, "fp64", [(37,), (300,), (2,)], True),
    (3, 1, "fp32", [(9, 8, 7), (20, 5, 3), (2, 2, 2)], False),
    (3, 2, "fp32_comp", [(12, 9, 5), (6, 6, 6)], False),
])
def test_batch_equals_per_plan_steps(d, m, prec, sizes, var):
    _say(f"[batch] d={d} m={m} {prec} shots={sizes} var={var}")
    rng = np.random.default_rng(len(sizes) + 10 * d + m)
    plans, states = _shots(d, m, prec, sizes, rng, var)
    ref = [(p.clone(), u.clone()) for p, u in states]
    batch = hl.Batch(plans)
    for n in (3, 20):                                   # eager, then graph replay + eager tail
        batch.step([p for p, _ in states], [u for _, u in states], n)
        for plan, (p, u) in zip(plans, ref):
            plan.step(p, u, n)
        torch.cuda.synchronize()
        for (p, u), (pr, ur) in zip(states, ref):
            assert torch.equal(p, pr) and torch.equal(u, ur)
    # new buffers: descriptors are rebuilt
    fresh = [(p.clone(), u.clone()) for p, u in states]
    batch.step([p for p, _ in fresh], [u for _, u in fresh], 2)
    for plan, (p, u) in zip(plans, ref):
        plan.step(p, u, 2)
    torch.cuda.synchronize()
    for (p, u), (pr, ur) in zip(fresh, ref):
        assert torch.equal(p, pr) and torch.equal(u, ur)
    batch.close()


def test_batch_rejects_mixed_problems():
    a = hl.Plan(2, 2, (8, 8))
    b = hl.Plan(2, 3, (8, 8))
    with pytest.raises(hl.HLError) as ei:
        hl.Batch([a, b])
    assert ei.value.status == hl.HL_ERR_ARG
    w = hl.Plan(2, 2, (8, 8), boundary="walls")
    with pytest.raises(hl.HLError) as ei:
        hl.Batch([a, w])
    assert ei.value.status == hl.HL_ERR_UNSUPPORTED
    c = hl.Plan(2, 2, (8, 8))
    k = inputs.kappa_sines(2, 2, (8, 8), (1.0, 1.0), (0.1, 0.1), (1, 1), "primal")
    c.set_kappa(k, k)
    batch = hl.Batch([a, c])
    pa, ua = a.alloc()
    pc, uc = c.alloc()
    with pytest.raises(hl.HLError) as ei:
        batch.step([pa, pc], [ua, uc], 1)
    assert ei.value.status == hl.HL_ERR_ARG
