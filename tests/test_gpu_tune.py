"""Launch shapes (hl_set_tile) and the tile autotuner (hl_tune): every tile
shape and 3D y-group computes each node with the same arithmetic, so steps must
be bit-identical to the default shape's, including ragged tiles at the grid's
edges; the tuner keeps one of its candidates and leaves (p, u) untouched."""

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


SHAPES = {1: [(256, 1, 0), (128, 1, 0), (64, 1, 0)],
          2: [(64, 4, 0), (64, 2, 0), (64, 1, 0), (128, 2, 0), (128, 1, 0), (256, 1, 0), (32, 8, 0), (32, 2, 0)],
          3: [(64, 4, 1), (64, 4, 4), (64, 2, 2), (128, 1, 1), (32, 8, 2), (256, 1, 4)]}


@pytest.mark.parametrize("d,m,K,prec,boundary", [
    (1, 3, (300,), "fp64", "periodic"),
    (2, 3, (130, 37), "fp32", "periodic"),
    (2, 2, (70, 21), "fp64", "walls"),
    (3, 2, (70, 9, 6), "fp32", "periodic"),
    (3, 1, (33, 17, 5), "fp32_comp", "walls"),
])
def test_every_tile_shape_gives_identical_steps(d, m, K, prec, boundary):
    _say(f"[tune] shapes d={d} m={m} K={K} {prec} {boundary}")
    rng = np.random.default_rng(40 + d + m)
    ref = hl.Plan(d, m, K, cfl=0.6, precision=prec, boundary=boundary)
    P0 = inputs.random_data(rng, d, m, ref.host_shapes()[0][:d])
    if boundary == "walls":
        P0 = inputs.zero_on_walls(P0, d)
    U0 = rng.uniform(-1, 1, ref.host_shapes()[1])
    p, u = ref.alloc()
    ref.init(p, u, P0, U0)
    p0, u0 = p.clone(), u.clone()
    ref.step(p, u, 5)
    for tx, ty, yg in SHAPES[d]:
        plan = hl.Plan(d, m, K, cfl=0.6, precision=prec, boundary=boundary)
        plan.set_tile(tx, ty, yg)
        assert (plan.info.tile[0], plan.info.tile[1]) == (tx, ty)
        q, v = p0.clone(), u0.clone()
        plan.step(q, v, 5)
        torch.cuda.synchronize()
        assert torch.equal(q, p) and torch.equal(v, u), (tx, ty, yg)
        plan.close()


def test_tune_keeps_a_candidate_and_the_state():
    _say("[tune] autotuner 2D m=3 (200, 96) fp32 and 3D m=1 (40, 24, 16) fp64")
    rng = np.random.default_rng(3)
    for d, m, K, prec in [(2, 3, (200, 96), "fp32"), (3, 1, (40, 24, 16), "fp64")]:
        plan = hl.Plan(d, m, K, cfl=0.5, precision=prec)
        p, u = plan.alloc()
        plan.init(p, u, inputs.random_data(rng, d, m, K), inputs.random_data(rng, d, m, K, ncomp=d))
        p0, u0 = p.clone(), u.clone()
        tx, ty, yg = plan.tune(p, u, reps=2)
        torch.cuda.synchronize()
        assert torch.equal(p, p0) and torch.equal(u, u0)
        assert (tx, ty) in [(s[0], s[1]) for s in SHAPES[d]] + [(64, 1), (128, 2), (32, 8)]
        ref = hl.Plan(d, m, K, cfl=0.5, precision=prec)
        q, v = p0.clone(), u0.clone()
        ref.step(q, v, 3)
        plan.step(p, u, 3)
        torch.cuda.synchronize()
        assert torch.equal(p, q) and torch.equal(u, v)


def test_set_tile_rejects_bad_shapes():
    plan = hl.Plan(2, 1, (16, 16))
    for tx, ty in [(48, 2), (16, 4), (64, 8), (512, 1), (32, 1)]:
        with pytest.raises(hl.HLError) as ei:
            plan.set_tile(tx, ty)
        assert ei.value.status == hl.HL_ERR_ARG
    p1 = hl.Plan(1, 1, (16,))
    with pytest.raises(hl.HLError):
        p1.set_tile(64, 2)


def test_batch_uses_the_shots_common_tile():
    """Shots tuned to one common shape are batched with it (bit-identical to
    their own steps); mixed shapes fall back to the default."""
    _say("[tune] batch with a common tile 2D m=3 fp32")
    rng = np.random.default_rng(21)
    for shapes in ([(256, 1, 0)] * 3, [(32, 8, 0), (128, 2, 0), (64, 4, 0)]):
        plans, states = [], []
        for K, (tx, ty, yg) in zip([(90, 40), (64, 33), (17, 70)], shapes):
            plan = hl.Plan(2, 3, K, cfl=0.5, precision="fp32")
            plan.set_tile(tx, ty, yg)
            p, u = plan.alloc()
            plan.init(p, u, inputs.random_data(rng, 2, 3, K), inputs.random_data(rng, 2, 3, K, ncomp=2))
            plans.append(plan)
            states.append((p, u))
        ref = [(p.clone(), u.clone()) for p, u in states]
        batch = hl.Batch(plans)
        batch.step([p for p, _ in states], [u for _, u in states], 18)
        for plan, (p, u) in zip(plans, ref):
            plan.step(p, u, 18)
        torch.cuda.synchronize()
        for (p, u), (pr, ur) in zip(states, ref):
            assert torch.equal(p, pr) and torch.equal(u, ur)
        batch.close()
