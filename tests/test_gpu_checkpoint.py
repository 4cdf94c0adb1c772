"""Checkpoint and resume: a run saved after n1 steps, restored into a fresh
plan made from the checkpoint's header and advanced n2 more steps equals the
uninterrupted run of n1 + n2 steps bit for bit; corrupted buffers and
mismatched plans are rejected."""

import sys

import numpy as np
import pytest

from paper_1808_10481_amd import checkpoint, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1808_10481_amd import hl  # noqa: E402


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("d,m,K,prec,boundary", [
    (3, 2, (24, 12, 10), "fp32", "periodic"),
    (2, 3, (70, 33), "fp64", "walls"),
    (3, 1, (16, 8, 9), "fp32_comp", "periodic"),
])
def test_resume_is_bitwise_identical(tmp_path, d, m, K, prec, boundary):
    _say(f"[checkpoint] d={d} m={m} K={K} {prec} {boundary}")
    n1, n2 = 7, 19
    plan = hl.Plan(d, m, K, cfl=0.5, precision=prec, boundary=boundary)
    rng = np.random.default_rng(3)
    P0 = inputs.random_data(rng, d, m, plan.host_shapes()[0][:d])
    if boundary == "walls":
        P0 = inputs.zero_on_walls(P0, d)
    p, u = plan.alloc()
    plan.init(p, u, P0, np.zeros(plan.host_shapes()[1]), startup=True)
    plan.step(p, u, n1)
    prefix = str(tmp_path / "state")
    checkpoint.save(plan, p, u, n1, prefix)
    plan.step(p, u, n2)
    torch.cuda.synchronize()

    h = checkpoint.read_header(prefix)
    assert h["step"] == n1
    plan2 = checkpoint.make_plan(h)
    q, v = plan2.alloc()
    assert checkpoint.restore(plan2, q, v, prefix) == n1
    plan2.step(q, v, n2)
    torch.cuda.synchronize()
    assert torch.equal(p, q) and torch.equal(u, v)

    # a plan with another time step is refused, and so is a corrupted buffer
    other = hl.Plan(d, m, K, cfl=0.4, precision=prec, boundary=boundary)
    with pytest.raises(ValueError):
        checkpoint.restore(other, q, v, prefix)
    other.close()
    raw = bytearray(open(prefix + ".u.bin", "rb").read())
    raw[len(raw) // 2] ^= 1
    open(prefix + ".u.bin", "wb").write(bytes(raw))
    with pytest.raises(ValueError):
        checkpoint.restore(plan2, q, v, prefix)
    plan.close()
    plan2.close()
