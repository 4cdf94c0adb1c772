"""Benchmark: Hermite-leapfrog cell-updates/s on one MI355X.

Workload: 2D periodic unit square, constant coefficient (kappa = 1), Hermite
order m = 3 (16 scaled coefficients per field per node), 1024 x 1024 cells,
nu = c dt / h = 0.5, seeded standing mode sin(2 pi k x) sin(2 pi l y)
(k, l in [1, 8]); the state starts resident in HBM.  A step is one pressure
half-step plus one velocity half-step over the whole grid (one cell-update
per node per step).  FP64 is the headline; FP32 is timed in the same run.

Prints one JSON line.  Run as: python bench.py [--steps K] [--warmup W].
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Hermite cell-updates/s (FP64 vs FP32) at stated L2 error; % HBM roofline"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_precision(hl, torch, wl, prec, steps, warmup):
    plan = hl.Plan(wl.d, wl.m, wl.K, dt=wl.dt, c=1.0, precision=prec)
    p, u = plan.alloc()
    plan.init(p, u, wl.P0, wl.U0)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.p_half(p, u)
        plan.u_half(u, p)
    # restart from the initial state so the timed run is the workload itself
    plan.init(p, u, wl.P0, wl.U0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for n in range(steps):
        plan.p_half(p, u)
        ev[2 * n + 1].record(stream)
        plan.u_half(u, p)
        ev[2 * n + 2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tp = [ev[2 * n].elapsed_time(ev[2 * n + 1]) for n in range(steps)]
    tu = [ev[2 * n + 1].elapsed_time(ev[2 * n + 2]) for n in range(steps)]
    total_ms = ev[0].elapsed_time(ev[-1])
    P, U = plan.export(p, u)
    info, word = plan.info, plan.coef_bytes
    plan.close()
    del p, u
    torch.cuda.empty_cache()
    return dict(total_ms=total_ms, wall_s=wall, p_ms=float(np.mean(tp)), u_ms=float(np.mean(tu)),
                P=P, U=U, word=word, nodes=info.nodes, nc=info.nc)


def _source_sha256():
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1808_10481_amd", "csrc", "*")))
    for f in files + [os.path.join(ROOT, "include", "hl.h")]:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def _profiled_traffic(kernel, prec, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this workload, or None when there is none or the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    try:
        rec = json.load(open(path))
    except OSError:
        return None
    if rec.get("source_sha256") != _source_sha256():
        return None
    return rec["kernels"].get(f"{kernel}_{prec}", {}).get("bytes_per_launch")


def roofline(res, d, prec="fp64", workload="standing_mode_2d_m3_1024"):
    """Dominant kernel: algorithmic HBM bytes per launch / average duration.
    p half-step reads u (d fields) and p, writes p: (d + 2) nc words per node;
    u half-step reads p and u, writes u: (2 d + 1) nc words per node."""
    per = {"p_half": ((d + 2) * res["nc"] * res["word"], res["p_ms"]),
           "u_half": ((2 * d + 1) * res["nc"] * res["word"], res["u_ms"])}
    name = max(per, key=lambda k: per[k][1])
    bpn, ms = per[name]
    gbs = bpn * res["nodes"] / (ms * 1e-3) / 1e9
    traffic = _profiled_traffic(name, prec, workload)
    out = {"kernel": name, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
           "algorithmic_bytes_per_launch": bpn * res["nodes"], "bytes_per_cell": bpn, "avg_ms": round(ms, 5)}
    if traffic:
        out["traffic_over_algorithmic"] = round(traffic / (bpn * res["nodes"]), 4)
    return out


def run_3d(hl, torch, steps, K=256, m=2):
    """3D m=2 256^3 Gaussian pulse (start-up from u = 0), FP32 bulk state:
    `steps` steps timed (the workload's 500 by default).  Reported beside the 2D
    headline with its own roofline (3D step: 12 (m+1)^3 coefficients read +
    written per half-step pair, p: 5 nc, u: 7 nc per node).  Every precision
    runs the same start-up, 3 untimed and `steps` timed steps; the pressure
    state is then compared with the FP64 run's."""
    from paper_1808_10481_amd import inputs
    wl = inputs.gaussian_pulse_3d(seed=2, K=K, m=m, steps=steps)
    res = {}
    finals = {}
    for prec in ("fp64", "fp32", "fp32_comp"):
        log(f"[bench] 3d {prec}: {steps} steps at {K}^3")
        plan = hl.Plan(3, m, wl.K, dt=wl.dt, c=1.0, precision=prec)
        p, u = plan.alloc()
        plan.init(p, u, wl.P0, None, startup=True)
        for _ in range(3):
            plan.p_half(p, u)
            plan.u_half(u, p)
        stream = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps + 1)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for n in range(steps):
            plan.p_half(p, u)
            ev[2 * n + 1].record(stream)
            plan.u_half(u, p)
            ev[2 * n + 2].record(stream)
        torch.cuda.synchronize()
        tp = float(np.mean([ev[2 * n].elapsed_time(ev[2 * n + 1]) for n in range(steps)]))
        tu = float(np.mean([ev[2 * n + 1].elapsed_time(ev[2 * n + 2]) for n in range(steps)]))
        total = ev[0].elapsed_time(ev[-1])
        info = plan.info
        r = {"nc": info.nc, "word": plan.coef_bytes, "nodes": info.nodes, "p_ms": tp, "u_ms": tu}
        step_bytes = 3 * 4 * info.nc * plan.coef_bytes * info.nodes
        res[prec] = {"value": wl.cells * steps / (total * 1e-3), "unit": "cell-updates/s",
                     "ms_per_step": total / steps, "steps": steps,
                     "step_hbm_frac": round(step_bytes / (total / steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "roofline": roofline(r, 3, prec, f"gaussian_pulse_3d_m{m}_{K}")}
        finals[prec] = plan.export(p, u, want_u=False)[0]
        if prec != "fp64":
            ref = finals["fp64"]
            res[prec]["rel_l2_vs_fp64_p_state"] = float(np.linalg.norm(finals[prec] - ref) / np.linalg.norm(ref))
            res[prec]["rel_l2_vs_fp64_p_nodal_values"] = float(
                np.linalg.norm(finals[prec][..., 0, 0, 0] - ref[..., 0, 0, 0]) / np.linalg.norm(ref[..., 0, 0, 0]))
            res[prec]["speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / res[prec]["ms_per_step"]
            del finals[prec]
        plan.close()
        del p, u
        torch.cuda.empty_cache()
    res["config"] = {"workload": f"gaussian_pulse_3d m={m} {K}^3 nu=0.5 width=0.05", "d": 3, "m": m,
                     "cells": [K] * 3}
    return res


def run_walls(hl, torch, steps, K=1024, m=3):
    """Walled 2D m=3 1024^2 Gaussian pulse (reflecting boundary, start-up from
    u = 0): `steps` steps timed after 3 untimed ones.  Each step is the ghost
    refresh, the pressure and the velocity half-step."""
    from paper_1808_10481_amd import inputs
    wl = inputs.gaussian_pulse_walls_2d(seed=3, K=K, m=m, steps=steps)
    res = {}
    for prec in ("fp64", "fp32"):
        log(f"[bench] walls 2d {prec}: {steps} steps at {K}^2")
        plan = hl.Plan(2, m, wl.K, length=wl.length, dt=wl.dt, c=1.0, precision=prec, boundary="walls")
        p, u = plan.alloc()
        plan.init(p, u, wl.P0, None, startup=True)
        plan.step(p, u, 3)
        stream = torch.cuda.current_stream()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record(stream)
        plan.step(p, u, steps)
        e.record(stream)
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / steps
        sp, su = plan.norms(p, u)
        res[prec] = {"value": (K + 1) ** 2 / (ms * 1e-3), "unit": "cell-updates/s", "ms_per_step": ms,
                     "steps": steps, "energy_like_sumsq": [sp, su]}
        plan.close()
        del p, u
        torch.cuda.empty_cache()
    res["config"] = {"workload": f"gaussian_pulse_walls_2d m={m} {K}^2 box [0,2]^2 nu=0.5 width^2=0.002",
                     "d": 2, "m": m, "cells": [K, K], "boundary": "walls"}
    return res


def run_varkappa(hl, torch, steps, K=1024, m=3):
    """Variable coefficient (per-node Taylor data of kappa), 2D m=3 FP32 on
    the largest grid of the batched-shot configuration (1024^2), smooth
    kappa = 1 + 0.35 sin(4 pi x) + 0.25 sin(6 pi y), standing-mode data:
    `steps` steps timed after 3 untimed ones, with the tile shape picked by
    the autotuner (hl_tune); FP64 beside it."""
    from paper_1808_10481_amd import inputs
    res = {}
    L = (1.0, 1.0)
    kp = inputs.kappa_sines(2, m, (K, K), L, (0.35, 0.25), (2, 3), "primal")
    ku = inputs.kappa_sines(2, m, (K, K), L, (0.35, 0.25), (2, 3), "dual")
    for prec in ("fp32", "fp64"):
        log(f"[bench] variable kappa 2d m={m} {K}^2 {prec}: {steps} steps")
        plan = hl.Plan(2, m, (K, K), cfl=0.5, c=float(np.sqrt(1.6)), precision=prec)
        plan.set_kappa(kp, ku)
        P0, U0 = inputs.standing_mode(2, m, (K, K), L, (3, 2), 0.0, plan.dt / 2)
        p, u = plan.alloc()
        plan.init(p, u, P0, U0)
        tile = plan.tune(p, u, reps=3)
        plan.step(p, u, 3)
        stream = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps + 1)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for n in range(steps):
            plan.p_half(p, u)
            ev[2 * n + 1].record(stream)
            plan.u_half(u, p)
            ev[2 * n + 2].record(stream)
        torch.cuda.synchronize()
        total = ev[0].elapsed_time(ev[-1])
        tp = float(np.mean([ev[2 * n].elapsed_time(ev[2 * n + 1]) for n in range(steps)]))
        tu = float(np.mean([ev[2 * n + 1].elapsed_time(ev[2 * n + 2]) for n in range(steps)]))
        res[prec] = {"value": K * K * steps / (total * 1e-3), "unit": "cell-updates/s", "ms_per_step": total / steps,
                     "p_half_ms": tp, "u_half_ms": tu, "steps": steps, "tile": list(tile)}
        plan.close()
        del p, u
        torch.cuda.empty_cache()
    res["config"] = {"workload": f"variable_kappa_2d m={m} {K}^2 kappa=1+0.35sin(4pi x)+0.25sin(6pi y), one shot, "
                                 "tuned tile", "d": 2, "m": m, "cells": [K, K]}
    return res


def run_batch(hl, torch, steps, nshots=32, m=3):
    """Batched shots: `nshots` periodic square grids with seeded sizes in
    [256, 1024] (the batched configuration's size mix), m=3 FP32, each with
    its own seeded layered medium c(y) in [1, 3] (three smoothed tanh steps,
    per-node kappa data on both grids) and a Ricker point source, starting at
    rest; `steps` steps advanced (a) with one launch per half-step for all
    shots (hl_batch_step, sources inside the batched step) and (b) shot by
    shot with hl_step (no source)."""
    from paper_1808_10481_amd import inputs
    rng = np.random.default_rng(6)
    sizes = [int(k) for k in rng.integers(256, 1025, nshots)]
    plans, states, media = [], [], []
    for K in sizes:
        up = rng.uniform(0.3, 1.0, 2)
        med = inputs.layered_speed(1.0, [up[0], up[1], -(up[0] + up[1])], np.sort(rng.uniform(0.15, 0.85, 3)),
                                   float(rng.uniform(0.02, 0.05)))
        cmax = 1.0 + up[0] + up[1]
        plan = hl.Plan(2, m, (K, K), cfl=0.5, c=float(cmax), precision="fp32")
        plan.set_kappa(inputs.kappa_layers(2, m, (K, K), (1.0, 1.0), med, "primal"),
                       inputs.kappa_layers(2, m, (K, K), (1.0, 1.0), med, "dual"))
        p, u = plan.alloc()
        p.zero_()
        u.zero_()
        plans.append(plan)
        states.append((p, u))
        media.append(med)
    cells = sum(K * K for K in sizes)
    batch = hl.Batch(plans)
    ps, us = [p for p, _ in states], [u for _, u in states]
    # a Ricker point source per shot (f0 seeded in [5, 15] cycles per unit
    # time, narrow Gaussian support of width 2 h at a seeded position), inside
    # the batched launch
    srcs, amps, nsrc = [], [], 0
    for plan, K in zip(plans, sizes):
        nodes, vals = inputs.point_source(2, m, (K, K), (1.0, 1.0), tuple(rng.uniform(0.2, 0.8, 2)), 2.0 / K)
        f0 = float(rng.uniform(5.0, 15.0))
        r = inputs.ricker(f0, 1.2 / f0)
        srcs.append((nodes, vals))
        amps.append(np.array([plan.dt * r((n + 0.5) * plan.dt) for n in range(steps + 32)]))
        nsrc += len(nodes)
    batch.set_sources(srcs, amps)
    batch.step(ps, us, 16)                                     # warm-up + graph capture
    for plan, (p, u) in zip(plans, states):
        plan.step(p, u, 16)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    batch.step(ps, us, steps)
    ev[1].record(stream)
    for plan, (p, u) in zip(plans, states):
        plan.step(p, u, steps)
    ev[2].record(stream)
    torch.cuda.synchronize()
    tb, ts = ev[0].elapsed_time(ev[1]) / steps, ev[1].elapsed_time(ev[2]) / steps
    batch.close()
    for plan in plans:
        plan.close()
    del states, ps, us
    torch.cuda.empty_cache()
    return {"batched": {"value": cells / (tb * 1e-3), "unit": "cell-updates/s", "ms_per_step": tb},
            "per_shot": {"value": cells / (ts * 1e-3), "unit": "cell-updates/s", "ms_per_step": ts},
            "speedup_batched_vs_per_shot": ts / tb, "steps": steps,
            "note": "per-shot stepping has no source term; the batched steps include the Ricker sources",
            "config": {"workload": f"batched_shots_2d {nshots} shots m={m} fp32, sizes seeded in [256, 1024]^2, "
                                   "layered c(y) in [1, 3] per shot (variable kappa), one Ricker point source per "
                                   "shot (f0 in [5, 15])",
                       "cells": cells, "sizes": sizes, "source_nodes": nsrc}}


def run_adjoint(hl, torch, steps, K=512, m=2):
    """Discrete adjoint on the shape of the gradient workload (2D, m=2, 512^2,
    periodic, constant kappa): `steps` transposed steps alone, then `steps`
    steps with the kappa gradient (forward state walked back by the reversed
    step, two inner products per step).  Forward steps timed beside them."""
    from paper_1808_10481_amd import inputs
    res = {}
    for prec in ("fp32", "fp64"):
        log(f"[bench] adjoint 2d m={m} {K}^2 {prec}: {steps} steps")
        rng = np.random.default_rng(4)
        plan = hl.Plan(2, m, (K, K), cfl=0.5, c=1.0, precision=prec)
        p, u = plan.alloc()
        pb, ub = plan.alloc()
        plan.init(p, u, inputs.random_data(rng, 2, m, (K, K)), inputs.random_data(rng, 2, m, (K, K), ncomp=2))
        plan.init(pb, ub, inputs.random_data(rng, 2, m, (K, K)), inputs.random_data(rng, 2, m, (K, K), ncomp=2))
        g = torch.zeros(1, dtype=torch.float64, device="cuda")
        plan.adjoint_step(pb, ub, 2, p=p, u=u, grad_kappa=g)     # warm-up, allocates the gradient buffers
        stream = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        plan.step(p, u, steps)
        ev[1].record(stream)
        plan.adjoint_step(pb, ub, steps)
        ev[2].record(stream)
        plan.adjoint_step(pb, ub, steps, p=p, u=u, grad_kappa=g)
        ev[3].record(stream)
        torch.cuda.synchronize()
        fwd, adj, grd = (ev[i].elapsed_time(ev[i + 1]) / steps for i in range(3))
        res[prec] = {"forward_ms_per_step": fwd, "adjoint_ms_per_step": adj, "gradient_ms_per_step": grd,
                     "adjoint_cell_updates_per_s": K * K / (adj * 1e-3), "steps": steps}
        plan.close()
        del p, u, pb, ub
        torch.cuda.empty_cache()
    res["config"] = {"workload": f"adjoint_2d m={m} {K}^2 periodic constant kappa", "d": 2, "m": m, "cells": [K, K]}
    return res


def run_kappa_gradient(hl, torch, steps, K=512, m=2, ndir=8):
    """Gradient of a receiver misfit with respect to the kappa data (2D, m=2,
    512^2, periodic, FP32): the "observed" traces come from a seeded smooth
    kappa, the model kappa is a seeded smooth perturbation of it; a Gaussian
    pulse (width 0.05, seeded centre) starts the wave, 16 receivers on a line
    record coefficient 0 of the pressure after every step.  Timed: forward
    with sqrt(N) checkpoints plus the checkpointed backward (segment re-runs
    and hl_adjoint_step_var per step).  Then the gradient's directional
    derivatives against fourth-order central differences of the same FP32
    forward on `ndir` random smooth directions."""
    from paper_1808_10481_amd import autograd as hag
    from paper_1808_10481_amd import inputs
    rng = np.random.default_rng(11)
    d, KK = 2, (K, K)
    log(f"[bench] kappa gradient 2d m={m} {K}^2 fp32: {steps} steps, sqrt(N) checkpoints")
    waves = tuple(int(w) for w in rng.integers(1, 4, d))
    amps_true = tuple(rng.uniform(0.15, 0.3, d))
    amps_model = tuple(a * rng.uniform(0.7, 0.9) for a in amps_true)
    kt = [inputs.kappa_sines(d, m, KK, (1.0, 1.0), amps_true, waves, g) for g in ("primal", "dual")]
    km = [inputs.kappa_sines(d, m, KK, (1.0, 1.0), amps_model, waves, g) for g in ("primal", "dual")]
    cmax = float(np.sqrt(1.0 + sum(amps_true)))
    plan = hl.Plan(d, m, KK, cfl=0.5, c=cmax, precision="fp32")
    p0, u0 = plan.alloc()
    centre = tuple(rng.uniform(0.3, 0.7, d))
    plan.init(p0, u0, inputs.gaussian_pulse(d, m, KK, (1.0, 1.0), centre, 0.05), np.zeros(plan.host_shapes()[1]))
    rec = [(int(x), K // 4) for x in np.linspace(K // 16, K - K // 16, 16)]
    with torch.no_grad():
        obs, _, _ = hag.receiver_traces(torch.tensor(kt[0]), torch.tensor(kt[1]), p0, u0, plan, steps, rec)
    obs = obs.double()

    def misfit(a, b, grad):
        with torch.set_grad_enabled(grad):
            tr, _, _ = hag.receiver_traces(a, b, p0, u0, plan, steps, rec)
            return 0.5 * ((tr.double() - obs) ** 2).sum()

    kp = torch.tensor(km[0], requires_grad=True)
    ku = torch.tensor(km[1], requires_grad=True)
    misfit(torch.tensor(km[0]), torch.tensor(km[1]), False)     # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = misfit(kp, ku, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    gp, gu = kp.grad.numpy(), ku.grad.numpy()
    decay = np.ones((2 * m + 2,) * d)
    for idx in np.ndindex(*decay.shape):
        decay[idx] = 0.5 ** sum(idx)
    errs = []
    eps = 2e-3
    for _ in range(ndir):
        dp = rng.normal(size=gp.shape) * decay
        du = rng.normal(size=gu.shape) * decay

        def L(s):
            return float(misfit(torch.tensor(km[0] + s * dp), torch.tensor(km[1] + s * du), False))

        fd = (-L(2 * eps) + 8 * L(eps) - 8 * L(-eps) + L(-2 * eps)) / (12 * eps)
        an = float(np.sum(gp * dp) + np.sum(gu * du))
        errs.append(abs(fd - an) / max(abs(fd), 1e-300))
    plan.close()
    del p0, u0
    torch.cuda.empty_cache()
    fwd_ms, bwd_ms = (t1 - t0) * 1e3, (t2 - t1) * 1e3
    seg = int(np.ceil(np.sqrt(steps)))
    log(f"[bench] kappa gradient: forward {fwd_ms:.1f} ms, backward {bwd_ms:.1f} ms, FD rel err max {max(errs):.2e}")
    return {"config": {"workload": f"kappa_gradient_2d m={m} {K}^2 periodic fp32, receiver misfit, "
                                   f"16 receivers, {steps} steps, sqrt(N) checkpoints", "d": d, "m": m,
                       "cells": [K, K], "steps": steps, "checkpoint_segment": seg},
            "misfit": float(loss.detach()), "forward_ms": fwd_ms, "backward_ms": bwd_ms,
            "ms_per_step_forward_plus_backward": (fwd_ms + bwd_ms) / steps,
            "gradient_cell_steps_per_s": K * K * steps / ((t2 - t0)),
            "fd_check": {"directions": ndir, "eps": eps, "rel_err": errs, "max_rel_err": max(errs),
                         "note": "fourth-order central differences of the FP32 forward"}}


def copy_probe(torch, nbytes=1 << 30, reps=20):
    """Plain device copy y <- x of nbytes (the paper's "realistic peak"
    vector-copy measurement); GB/s counts bytes read + written."""
    x = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        y.copy_(x)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del x, y
    torch.cuda.empty_cache()
    return {"bytes_moved": 2 * nbytes, "avg_ms": round(ms, 4), "gbs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


def cpu_baseline(wl, rows):
    """The oracle, as it stands, on one step over the nodes of `rows` grid rows."""
    import oracle
    prob = oracle.Problem(wl.d, wl.m, wl.K, wl.length, wl.dt, 1.0)
    K0 = wl.K[0]
    nodes = np.stack(np.meshgrid(np.arange(K0), np.arange(rows), indexing="ij"), -1).reshape(-1, 2)
    t0 = time.perf_counter()
    Pn = oracle.p_half(prob, wl.P0, wl.U0, nodes=nodes)
    # the u half-step at these dual nodes needs the new P on their corners
    # (rows 0..rows); compute that extra row and splice it in
    P1 = np.array(wl.P0, copy=True)
    P1[:, :rows] = Pn.reshape(K0, rows, *Pn.shape[1:])
    extra = np.stack(np.meshgrid(np.arange(K0), np.array([rows % wl.K[1]]), indexing="ij"), -1).reshape(-1, 2)
    P1[:, rows % wl.K[1]] = oracle.p_half(prob, wl.P0, wl.U0, nodes=extra).reshape(K0, *Pn.shape[1:])
    Un = oracle.u_half(prob, wl.U0, P1, nodes=nodes)
    sec = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = 1
    return dict(value=nodes.shape[0] / sec, seconds=sec, cores=cores, P=Pn, U=Un, rows=rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--K", type=int, default=1024)
    ap.add_argument("--cpu-rows", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-comp", action="store_true")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--steps-3d", type=int, default=500)
    ap.add_argument("--no-walls", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-varkappa", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--steps-batch", type=int, default=2000)
    ap.add_argument("--steps-varkappa", type=int, default=50)
    ap.add_argument("--steps-adjoint", type=int, default=100)
    ap.add_argument("--no-kgrad", action="store_true")
    ap.add_argument("--steps-kgrad", type=int, default=2000)
    ap.add_argument("--steps-walls", type=int, default=200)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the build has no "
                          "multi-GPU path (see the sharding note in DESIGN.md)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_1808_10481_amd import hl, inputs
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    log(f"[bench] building workload standing_mode_2d K={args.K} m=3")
    wl = inputs.standing_mode_2d(seed=1, K=args.K, m=3, steps=args.steps)
    t_end = args.steps * wl.dt
    Pex, _ = inputs.standing_mode(2, 3, wl.K, wl.length, wl.waves, t_end, 0.0)
    vol = float(np.prod(wl.h))

    log(f"[bench] fp64: {args.warmup} warmup + {args.steps} timed steps")
    r64 = run_precision(hl, torch, wl, "fp64", args.steps, args.warmup)
    value64 = wl.cells * args.steps / (r64["total_ms"] * 1e-3)
    err64 = float(np.sqrt(vol * np.sum((r64["P"][..., 0, 0] - Pex[..., 0, 0]) ** 2)))
    log(f"[bench] fp64 {r64['total_ms'] / args.steps:.4f} ms/step, p {r64['p_ms']:.4f} u {r64['u_ms']:.4f} ms")

    out = {
        "metric": METRIC, "value": value64, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["total_ms"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"standing_mode_2d m=3 {args.K}x{args.K} nu=0.5 kappa=1 "
                               f"waves={list(wl.waves)}", "d": 2, "m": 3, "cells": list(wl.K),
                   "steps": args.steps, "parallelism": "single_gpu"},
        "roofline": roofline(r64, 2, "fp64"),
        "l2": {"fp64_nodal_vs_exact": err64},
    }

    if not args.no_fp32:
        log(f"[bench] fp32: {args.warmup} warmup + {args.steps} timed steps")
        r32 = run_precision(hl, torch, wl, "fp32", args.steps, args.warmup)
        value32 = wl.cells * args.steps / (r32["total_ms"] * 1e-3)
        den = np.sqrt(np.sum(r64["P"] ** 2) + np.sum(r64["U"] ** 2))
        rel = float(np.sqrt(np.sum((r32["P"] - r64["P"]) ** 2) + np.sum((r32["U"] - r64["U"]) ** 2)) / den)
        err32 = float(np.sqrt(vol * np.sum((r32["P"][..., 0, 0] - Pex[..., 0, 0]) ** 2)))
        v32 = np.concatenate([r32["P"][..., 0, 0].ravel(), r32["U"][..., 0, 0].ravel()])
        v64 = np.concatenate([r64["P"][..., 0, 0].ravel(), r64["U"][..., 0, 0].ravel()])
        relv = float(np.linalg.norm(v32 - v64) / np.linalg.norm(v64))
        out["fp32"] = {"value": value32, "ms_per_step": r32["total_ms"] / args.steps,
                       "rel_l2_vs_fp64_state": rel, "rel_l2_vs_fp64_nodal_values": relv,
                       "nodal_l2_vs_exact": err32,
                       "roofline": roofline(r32, 2, "fp32"), "speedup_vs_fp64": value32 / value64}
        log(f"[bench] fp32 {r32['total_ms'] / args.steps:.4f} ms/step, rel L2 vs fp64 {rel:.3e}")

    if not args.no_comp:
        log(f"[bench] fp32_comp: {args.warmup} warmup + {args.steps} timed steps")
        rc = run_precision(hl, torch, wl, "fp32_comp", args.steps, args.warmup)
        valuec = wl.cells * args.steps / (rc["total_ms"] * 1e-3)
        den = np.sqrt(np.sum(r64["P"] ** 2) + np.sum(r64["U"] ** 2))
        rel = float(np.sqrt(np.sum((rc["P"] - r64["P"]) ** 2) + np.sum((rc["U"] - r64["U"]) ** 2)) / den)
        vc = np.concatenate([rc["P"][..., 0, 0].ravel(), rc["U"][..., 0, 0].ravel()])
        v64 = np.concatenate([r64["P"][..., 0, 0].ravel(), r64["U"][..., 0, 0].ravel()])
        out["fp32_comp"] = {"value": valuec, "ms_per_step": rc["total_ms"] / args.steps,
                            "storage": "FP32 hi + BF16 lo (6 B/coefficient), FP64 arithmetic",
                            "rel_l2_vs_fp64_state": rel,
                            "rel_l2_vs_fp64_nodal_values": float(np.linalg.norm(vc - v64) / np.linalg.norm(v64)),
                            "nodal_l2_vs_exact": float(np.sqrt(vol * np.sum((rc["P"][..., 0, 0] - Pex[..., 0, 0]) ** 2))),
                            "roofline": roofline(rc, 2, "fp32_comp"), "speedup_vs_fp64": valuec / value64}
        log(f"[bench] fp32_comp {rc['total_ms'] / args.steps:.4f} ms/step, rel L2 vs fp64 {rel:.3e}")

    if not args.no_3d:
        out["gaussian_pulse_3d"] = run_3d(hl, torch, args.steps_3d)

    if not args.no_walls:
        out["gaussian_pulse_walls_2d"] = run_walls(hl, torch, args.steps_walls)

    if not args.no_varkappa:
        out["variable_kappa_2d"] = run_varkappa(hl, torch, args.steps_varkappa)

    if not args.no_batch:
        out["batched_shots_2d"] = run_batch(hl, torch, args.steps_batch)

    if not args.no_adjoint:
        out["adjoint_2d"] = run_adjoint(hl, torch, args.steps_adjoint)

    if not args.no_kgrad:
        out["kappa_gradient_2d"] = run_kappa_gradient(hl, torch, args.steps_kgrad)

    if not args.no_copy_probe:
        out["copy_probe"] = copy_probe(torch)
        log(f"[bench] copy probe {out['copy_probe']}")

    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle, one step over {args.cpu_rows} of {args.K} rows")
        cb = cpu_baseline(wl, args.cpu_rows)
        # parity of the same sample against one GPU FP64 step
        plan = hl.Plan(wl.d, wl.m, wl.K, dt=wl.dt, c=1.0, precision="fp64")
        p, u = plan.alloc()
        plan.init(p, u, wl.P0, wl.U0)
        plan.step(p, u, 1)
        P1, U1 = plan.export(p, u)
        plan.close()
        gp = P1[:, :args.cpu_rows].reshape(cb["P"].shape)
        gu = np.stack([U1[i][:, :args.cpu_rows].reshape(cb["P"].shape) for i in range(2)])
        num = np.sqrt(np.sum((gp - cb["P"]) ** 2) + np.sum((gu - cb["U"]) ** 2))
        den = np.sqrt(np.sum(cb["P"] ** 2) + np.sum(cb["U"] ** 2))
        out["l2"]["fp64_vs_oracle_one_step_sample"] = float(num / den)
        out["cpu_baseline"] = {"value": cb["value"], "unit": "cell-updates/s", "cores": cb["cores"],
                               "kind": "oracle",
                               "sample": f"one step (p and u half-steps) over the {args.K * args.cpu_rows} "
                                         f"nodes of {args.cpu_rows} of {args.K} rows, "
                                         f"{cb['seconds']:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
