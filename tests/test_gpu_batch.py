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


def _shots(d, m, prec, sizes, rng, var=False, walls=()):
    plans, states = [], []
    for i, K in enumerate(sizes):
        c = float(rng.uniform(0.8, 1.8))
        bc = "walls" if i in walls else "periodic"
        plan = hl.Plan(d, m, K, cfl=float(rng.uniform(0.3, 0.9)), c=c, precision=prec, boundary=bc)
        if var:
            amps = tuple(rng.uniform(0.05, 0.2, d))
            if bc == "walls":
                plan.set_kappa(inputs.kappa_box(d, m, K, (1.0,) * d, amps, "primal"),
                               inputs.kappa_box(d, m, K, (1.0,) * d, amps, "dual"))
            else:
                waves = tuple(int(w) for w in rng.integers(1, 3, d))
                plan.set_kappa(inputs.kappa_sines(d, m, K, (1.0,) * d, amps, waves, "primal"),
                               inputs.kappa_sines(d, m, K, (1.0,) * d, amps, waves, "dual"))
        p, u = plan.alloc()
        ps, us = plan.host_shapes()
        plan.init(p, u, inputs.random_data(rng, d, m, ps[:d]), inputs.random_data(rng, d, m, K, ncomp=d))
        plans.append(plan)
        states.append((p, u))
    return plans, states


@pytest.mark.parametrize("d,m,prec,sizes,var,walls", [
    (2, 3, "fp32", [(64, 48), (100, 37), (33, 80), (128, 128), (2, 3)], False, ()),
    (2, 2, "fp64", [(40, 24), (17, 9), (64, 64)], True, ()),
    (1, 5, "fp64", [(37,), (300,), (2,)], True, ()),
    (3, 1, "fp32", [(9, 8, 7), (20, 5, 3), (2, 2, 2)], False, ()),
    (3, 1, "fp64", [(9, 8, 7), (20, 5, 3)], True, ()),
    (3, 2, "fp32_comp", [(12, 9, 5), (6, 6, 6)], False, ()),
    (2, 3, "fp32", [(64, 48), (100, 37), (33, 20)], False, (0, 2)),
    (2, 2, "fp64", [(40, 24), (17, 9)], True, (1,)),
    (3, 1, "fp32_comp", [(12, 9, 5), (6, 7, 4)], False, (0, 1)),
    (2, 3, "fp32_comp", [(40, 24), (17, 9)], True, (1,)),
    (3, 2, "fp32", [(9, 8, 7), (6, 5, 4), (2, 2, 2)], True, ()),
    (3, 2, "fp64", [(6, 5, 4), (5, 4, 3)], True, (1,)),
    (3, 3, "fp32_comp", [(4, 3, 3), (3, 3, 2)], True, ()),
])
def test_batch_equals_per_plan_steps(d, m, prec, sizes, var, walls):
    _say(f"[batch] d={d} m={m} {prec} shots={sizes} var={var} walls={walls}")
    rng = np.random.default_rng(len(sizes) + 10 * d + m)
    plans, states = _shots(d, m, prec, sizes, rng, var, walls)
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


def test_batch_follows_member_kappa_and_tile_changes():
    """A member plan's hl_set_kappa (free + new buffers) or hl_set_tile between
    two batched steps on the same buffers: the batch rebuilds its
    descriptors and stays bit-identical to per-plan stepping."""
    _say("[batch] kappa/tile changes of a member between batched steps")
    d, m, sizes = 2, 2, [(40, 24), (17, 9)]
    rng = np.random.default_rng(77)
    plans, states = _shots(d, m, "fp64", sizes, rng, var=True)
    ref = [(p.clone(), u.clone()) for p, u in states]
    batch = hl.Batch(plans)

    def both(n):
        batch.step([p for p, _ in states], [u for _, u in states], n)
        for plan, (p, u) in zip(plans, ref):
            plan.step(p, u, n)
        torch.cuda.synchronize()
        for (p, u), (pr, ur) in zip(states, ref):
            assert torch.equal(p, pr) and torch.equal(u, ur)

    both(17)                                            # graph + eager tail
    K = sizes[1]
    kp = inputs.kappa_sines(d, m, K, (1.0,) * d, (0.15, 0.1), (2, 1), "primal")
    ku = inputs.kappa_sines(d, m, K, (1.0,) * d, (0.15, 0.1), (2, 1), "dual")
    plans[1].set_kappa(None, None)                      # frees the member's kappa buffers
    plans[1].set_kappa(kp, ku)                          # new buffers, new data
    both(17)
    plans[0].set_tile(128, 2, 0)
    plans[1].set_tile(128, 2, 0)                        # common tile: the batch launches it
    both(3)
    batch.close()


def test_batch_rejects_mixed_problems():
    a = hl.Plan(2, 2, (8, 8))
    b = hl.Plan(2, 3, (8, 8))
    with pytest.raises(hl.HLError) as ei:
        hl.Batch([a, b])
    assert ei.value.status == hl.HL_ERR_ARG
    c = hl.Plan(2, 2, (8, 8))
    k = inputs.kappa_sines(2, 2, (8, 8), (1.0, 1.0), (0.1, 0.1), (1, 1), "primal")
    c.set_kappa(k, k)
    batch = hl.Batch([a, c])
    pa, ua = a.alloc()
    pc, uc = c.alloc()
    with pytest.raises(hl.HLError) as ei:
        batch.step([pa, pc], [ua, uc], 1)
    assert ei.value.status == hl.HL_ERR_ARG


def _ricker(f0, t0, t_stop):
    """Ricker wavelet r(t) = (1 - 2 a) exp(-a), a = (pi f0 (t - t0))^2, cut to
    zero after t_stop."""
    def r(t):
        if t > t_stop:
            return 0.0
        a = (np.pi * f0 * (t - t0)) ** 2
        return (1.0 - 2.0 * a) * np.exp(-a)
    return r


def _point_source(d, m, K, centre, width):
    """A narrow Gaussian g as scaled data, kept on the nodes where it is not
    negligible: (node tuples, their data, the dense array with zeros elsewhere)."""
    G = inputs.gaussian_pulse(d, m, K, (1.0,) * d, centre, width)
    mag = np.abs(G).reshape(G.shape[:d] + (-1,)).max(-1)
    mask = mag > 1e-12 * mag.max()
    Gs = np.zeros_like(G)
    Gs[mask] = G[mask]
    return np.argwhere(mask), G[mask], Gs


@pytest.mark.parametrize("d,m,prec,sizes,var", [
    (2, 2, "fp64", [(40, 24), (17, 9), (64, 64)], True),
    (1, 3, "fp32", [(37,), (120,), (2,)], False),
    (2, 3, "fp32", [(64, 48), (100, 37), (5, 3)], False),
    (2, 2, "fp32_comp", [(40, 24), (17, 9)], True),
])
def test_batch_sources_equal_per_plan_steps_and_oracle(d, m, prec, sizes, var):
    """Sources inside the batched launch: bit-identical to each plan's own
    pressure half-step, hl_add_source of the dense g and velocity half-step;
    the FP64 case also against the oracle's midpoint-rule source step.
    FP32_COMP compares the stored values: the dense add rewrites every entry,
    and an entry whose lo word is exactly half an FP32 ulp may come back with
    its hi word rounded to even and the opposite lo (the same value)."""
    import oracle
    from tolerances import _close, tol
    _say(f"[batch] sources d={d} m={m} {prec} shots={sizes} var={var}")
    rng = np.random.default_rng(77 + 10 * d + m)
    plans, states, kap, srcs, dense, amps, rs = [], [], [], [], [], [], []
    namps, total = 26, 28
    for K in sizes:
        plan = hl.Plan(d, m, K, cfl=float(rng.uniform(0.3, 0.9)), c=float(rng.uniform(0.8, 1.8)), precision=prec)
        kk = None
        if var:
            a = tuple(rng.uniform(0.05, 0.2, d))
            w = tuple(int(x) for x in rng.integers(1, 3, d))
            kk = (inputs.kappa_sines(d, m, K, (1.0,) * d, a, w, "primal"),
                  inputs.kappa_sines(d, m, K, (1.0,) * d, a, w, "dual"))
            plan.set_kappa(*kk)
        p, u = plan.alloc()
        plan.init(p, u, inputs.random_data(rng, d, m, K) * 0.1, inputs.random_data(rng, d, m, K, ncomp=d) * 0.1)
        nodes, vals, Gs = _point_source(d, m, K, tuple(rng.uniform(0.2, 0.8, d)), 2.5 / max(K))
        f0 = float(rng.uniform(5.0, 15.0))
        r = _ricker(f0, 1.2 / f0, namps * plan.dt)
        plans.append(plan)
        states.append((p, u))
        kap.append(kk)
        srcs.append((nodes, vals))
        dense.append(Gs)
        rs.append(r)
        amps.append(np.array([plan.dt * r((n + 0.5) * plan.dt) for n in range(namps)]))
    init = [plan.export(p, u) for plan, (p, u) in zip(plans, states)]
    ref = [(p.clone(), u.clone()) for p, u in states]
    gbuf = [plan.source_buffer(G) for plan, G in zip(plans, dense)]
    batch = hl.Batch(plans)
    batch.set_sources(srcs, amps)
    t = 0
    for n in (3, 20, 5):                      # eager, graph replay + tail, past the last amplitude
        batch.step([p for p, _ in states], [u for _, u in states], n)
        for k in range(n):
            for i, (plan, (p, u)) in enumerate(zip(plans, ref)):
                plan.p_half(p, u)
                if t + k < namps:
                    plan.add_source(p, gbuf[i], amps[i][t + k])
                plan.u_half(u, p)
        t += n
        torch.cuda.synchronize()
        for plan, (p, u), (pr, ur) in zip(plans, states, ref):
            if prec == "fp32_comp":
                got, want = plan.export(p, u), plan.export(pr, ur)
                assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
            else:
                assert torch.equal(p, pr) and torch.equal(u, ur)
    assert t == total
    if prec == "fp64":
        for i in range(len(plans)):
            plan = plans[i]
            prob = oracle.Problem(d, m, tuple(sizes[i]), (1.0,) * d, plan.dt, plan.kappa)
            kw = {} if kap[i] is None else {"Kp": kap[i][0], "Ku": kap[i][1]}
            if kap[i] is not None:
                prob = oracle.Problem(d, m, tuple(sizes[i]), (1.0,) * d, plan.dt, 1.0)
            Po, Uo = oracle.step_with_source(prob, init[i][0], init[i][1], dense[i], rs[i], 0.0, total, **kw)
            Pg, Ug = plan.export(*states[i])
            _close(Pg, Po, *tol("fp64", d, m))
            _close(Ug, Uo, *tol("fp64", d, m))
    batch.set_sources(None)                    # removed: plain batched steps again
    batch.step([p for p, _ in states], [u for _, u in states], 2)
    for plan, (p, u) in zip(plans, ref):
        plan.step(p, u, 2)
    torch.cuda.synchronize()
    for plan, (p, u), (pr, ur) in zip(plans, states, ref):
        if prec == "fp32_comp":
            got, want = plan.export(p, u), plan.export(pr, ur)
            assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
        else:
            assert torch.equal(p, pr) and torch.equal(u, ur)
    batch.close()


def test_batch_sources_reject_bad_input():
    a = hl.Plan(2, 1, (8, 6), precision="fp32")
    batch = hl.Batch([a])
    nodes = np.array([[1, 2], [1, 2]])
    with pytest.raises(hl.HLError) as ei:
        batch.set_sources([(nodes, np.ones((2, 2, 2)))], [np.ones(3)])
    assert ei.value.status == hl.HL_ERR_ARG
    batch.close()


def test_batch_sources_on_walled_shots_equal_per_plan_steps():
    """Walled shots with sources in one batch: the per-shot ghost refresh, the
    batched half-steps and the source launch equal each plan's own steps."""
    _say("[batch] walled shots with sources 2D m=2 fp64")
    d, m = 2, 2
    rng = np.random.default_rng(515)
    plans, states = _shots(d, m, "fp64", [(30, 22), (17, 40)], rng, False, (0, 1))
    srcs, gbuf, amps = [], [], []
    for plan in plans:
        K = plan.cells
        G = inputs.gaussian_pulse(d, m, tuple(k + 1 for k in K), (1.0,) * d, tuple(rng.uniform(0.3, 0.7, d)),
                                  3.0 / max(K))
        mag = np.abs(G).reshape(G.shape[:d] + (-1,)).max(-1)
        mask = mag > 1e-12 * mag.max()
        Gs = np.zeros_like(G)
        Gs[mask] = G[mask]
        srcs.append((np.argwhere(mask), G[mask]))
        gbuf.append(plan.source_buffer(Gs))
        amps.append(rng.normal(size=24) * plan.dt)
    ref = [(p.clone(), u.clone()) for p, u in states]
    batch = hl.Batch(plans)
    batch.set_sources(srcs, amps)
    batch.step([p for p, _ in states], [u for _, u in states], 20)
    for n in range(20):
        for i, (plan, (p, u)) in enumerate(zip(plans, ref)):
            plan.p_half(p, u)
            plan.add_source(p, gbuf[i], amps[i][n])
            plan.u_half(u, p)
    torch.cuda.synchronize()
    for (p, u), (pr, ur) in zip(states, ref):
        assert torch.equal(p, pr) and torch.equal(u, ur)
    batch.close()
