"""Benchmark: Hermite-leapfrog cell-updates/s on one MI355X.

Headline workload: 3D periodic unit cube, constant coefficient (kappa = 1),
Hermite order m = 2 (27 scaled coefficients per field per node), 256^3
cells, nu = c dt / h = 0.5, Gaussian pressure pulse exp(-|x - x0|^2 / w^2),
w = 0.05, at a seeded centre (minimum image), u = 0 at t = 0 and the start-up
to dt/2; 500 steps timed with the state resident in HBM.  A step is one
pressure half-step plus one velocity half-step over the whole grid (one
cell-update per node per step).  FP64, the paper's precision, is the headline
`value`; FP32 and FP32_COMP run the same steps in the same invocation, each
with its roofline, its error against the FP64 run and the FP64 run's error
against the exact solution.  The other workloads (the 2D standing mode, 1D
standing wave, walls, variable kappa, batched shots, adjoint and kappa
gradient) follow as extra records, each with its own error statement.

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


def _rel_state(a, b):
    """Relative L2 of state a = (P, U) against b over all coefficients."""
    num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(a, b))
    den = sum(float(np.sum(y ** 2)) for y in b)
    return float(np.sqrt(num / den))


# The sources the profiled half-step kernels are compiled from: their code
# (hl_kernels.hpp), the table layout and storage policies they use, and the
# translation units that instantiate them.  A traffic record stays valid while
# these are unchanged.
KERNEL_SOURCES = ("hl_kernels.hpp", "hl_layout.hpp", "hl_storage.hpp", "hl_kernels_d2_fp64.hip",
                  "hl_kernels_d2_fp32.hip", "hl_kernels_d2_comp.hip", "hl_kernels_d3_fp64.hip",
                  "hl_kernels_d3_fp32.hip", "hl_kernels_d3_comp.hip")


def _source_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(name.encode())
        h.update(open(os.path.join(ROOT, "paper_1808_10481_amd", "csrc", name), "rb").read())
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


def _time_half_steps(plan, torch, p, u, steps):
    """`steps` steps, one event after each half-step on the launch stream;
    returns (total ms, mean p half-step ms, mean u half-step ms)."""
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
    return ev[0].elapsed_time(ev[-1]), tp, tu


def _exact_planes_3d(wl, t, planes):
    """Exact nodal pressure of the pulse on the primal nodes of z-planes
    `planes` (host layout [x][y][z_sel])."""
    from paper_1808_10481_amd import inputs
    K, h = wl.K[0], wl.h[0]
    x = np.arange(K) * h
    X = np.stack(np.meshgrid(x, x, np.asarray(planes) * h, indexing="ij"), -1)
    return inputs.pulse_exact_3d(X, wl.center, 0.05, t)


def run_3d(hl, torch, steps, K=256, m=2, sample=None, warmup=3):
    """3D m=2 256^3 Gaussian pulse (start-up from u = 0) in FP64, FP32 and
    FP32_COMP: start-up, `warmup` untimed and `steps` timed steps each.  Per
    precision: cell-updates/s, per-half-step times and the roofline of the
    slower half-step (p: (d+2) nc, u: (2d+1) nc words per node).  Errors: the
    FP64 run's nodal values against the exact solution (spherical means over
    periodic images) on every 16th z-plane; FP32 and FP32_COMP against the
    FP64 run (whole pressure state and nodal values).  `sample`: the CPU
    baseline's oracle results, compared with the FP64 state after the
    start-up and one step."""
    from paper_1808_10481_amd import inputs
    wl = inputs.gaussian_pulse_3d(seed=2, K=K, m=m, steps=steps)
    res = {}
    finals = {}
    t_end = (steps + warmup) * wl.dt
    planes = np.arange(0, K, 16)
    for prec in ("fp64", "fp32", "fp32_comp"):
        log(f"[bench] 3d {prec}: {steps} steps at {K}^3")
        plan = hl.Plan(3, m, wl.K, dt=wl.dt, c=1.0, precision=prec)
        p, u = plan.alloc()
        if prec == "fp64" and sample is not None:
            plan.init(p, u, wl.P0, None, startup=True)
            plan.step(p, u, 1)
            P1, U1 = plan.export(p, u)
            res["oracle_parity"] = sample_parity(sample, P1, U1)
            log(f"[bench] 3d fp64 vs oracle on the CPU sample: {res['oracle_parity']}")
            del P1, U1
        plan.init(p, u, wl.P0, None, startup=True)
        for _ in range(warmup):
            plan.p_half(p, u)
            plan.u_half(u, p)
        total, tp, tu = _time_half_steps(plan, torch, p, u, steps)
        info = plan.info
        r = {"nc": info.nc, "word": plan.coef_bytes, "nodes": info.nodes, "p_ms": tp, "u_ms": tu}
        step_bytes = 3 * 4 * info.nc * plan.coef_bytes * info.nodes
        res[prec] = {"value": wl.cells * steps / (total * 1e-3), "unit": "cell-updates/s",
                     "ms_per_step": total / steps, "steps": steps, "p_half_ms": tp, "u_half_ms": tu,
                     "step_hbm_frac": round(step_bytes / (total / steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "roofline": roofline(r, 3, prec, f"gaussian_pulse_3d_m{m}_{K}")}
        finals[prec] = plan.export(p, u, want_u=False)[0]
        if prec == "fp64":
            ex = _exact_planes_3d(wl, t_end, planes)
            got = finals["fp64"][:, :, planes, 0, 0, 0]
            res["fp64"]["nodal_rel_l2_vs_exact"] = float(np.linalg.norm(got - ex) / np.linalg.norm(ex))
            res["fp64"]["nodal_l2_vs_exact"] = float(np.sqrt(np.prod(wl.h) * K / len(planes)
                                                             * np.sum((got - ex) ** 2)))
        else:
            ref = finals["fp64"]
            res[prec]["rel_l2_vs_fp64_p_state"] = float(np.linalg.norm(finals[prec] - ref) / np.linalg.norm(ref))
            nv = float(np.linalg.norm(finals[prec][..., 0, 0, 0] - ref[..., 0, 0, 0])
                       / np.linalg.norm(ref[..., 0, 0, 0]))
            res[prec]["rel_l2_vs_fp64_p_nodal_values"] = nv
            disc = res["fp64"]["nodal_rel_l2_vs_exact"]
            res[prec]["adequate"] = bool(nv <= 0.1 * disc)
            res[prec]["speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / res[prec]["ms_per_step"]
            del finals[prec]
        log(f"[bench] 3d {prec}: {total / steps:.4f} ms/step (p {tp:.4f}, u {tu:.4f})")
        plan.close()
        del p, u
        torch.cuda.empty_cache()
    res["config"] = {"workload": f"gaussian_pulse_3d m={m} {K}^3 nu=0.5 width=0.05", "d": 3, "m": m,
                     "cells": [K] * 3, "t_end": t_end,
                     "exact_solution": "spherical means over periodic images, nodal values on every 16th z-plane",
                     "adequacy_rule": "round-off vs FP64 <= 0.1 x FP64 discretization error (relative, nodal)"}
    return res


def run_2d(hl, torch, steps, warmup, K=1024, mall_copy=None):
    """2D m=3 1024^2 standing mode (exact U at dt/2): FP64, FP32 and FP32_COMP,
    `steps` timed steps each after `warmup` untimed ones (restarted from the
    initial state).  Errors: nodal L2 against the exact solution per
    precision, and FP32/FP32_COMP against FP64 over the whole state.  The
    FP32 state (201 MB) fits in the 256 MB MALL, so its half-steps are also
    stated against a copy of a MALL-resident buffer (`mall_copy` GB/s)."""
    from paper_1808_10481_amd import inputs
    wl = inputs.standing_mode_2d(seed=1, K=K, m=3, steps=steps)
    Pex, _ = inputs.standing_mode(2, 3, wl.K, wl.length, wl.waves, steps * wl.dt, 0.0)
    vol = float(np.prod(wl.h))
    out = {}
    ref = None
    for prec in ("fp64", "fp32", "fp32_comp"):
        log(f"[bench] 2d {prec}: {warmup} warmup + {steps} timed steps")
        r = run_precision(hl, torch, wl, prec, steps, warmup)
        rec = {"value": wl.cells * steps / (r["total_ms"] * 1e-3), "unit": "cell-updates/s",
               "ms_per_step": r["total_ms"] / steps, "p_half_ms": r["p_ms"], "u_half_ms": r["u_ms"],
               "nodal_l2_vs_exact": float(np.sqrt(vol * np.sum((r["P"][..., 0, 0] - Pex[..., 0, 0]) ** 2))),
               "roofline": roofline(r, 2, prec)}
        if ref is None:
            ref = r
        else:
            den = np.sqrt(np.sum(ref["P"] ** 2) + np.sum(ref["U"] ** 2))
            rec["rel_l2_vs_fp64_state"] = float(np.sqrt(np.sum((r["P"] - ref["P"]) ** 2)
                                                        + np.sum((r["U"] - ref["U"]) ** 2)) / den)
            v = np.concatenate([r["P"][..., 0, 0].ravel(), r["U"][..., 0, 0].ravel()])
            v64 = np.concatenate([ref["P"][..., 0, 0].ravel(), ref["U"][..., 0, 0].ravel()])
            rec["rel_l2_vs_fp64_nodal_values"] = float(np.linalg.norm(v - v64) / np.linalg.norm(v64))
            rec["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / rec["ms_per_step"]
            rec["adequate"] = bool(rec["nodal_l2_vs_exact"] <= 1.1 * out["fp64"]["nodal_l2_vs_exact"])
        if prec == "fp32_comp":
            rec["storage"] = "FP32 hi + BF16 lo (6 B/coefficient), FP64 arithmetic"
        if prec == "fp32" and mall_copy:
            ach = rec["roofline"]["achieved"]
            rec["roofline"]["mall_resident"] = True
            rec["roofline"]["mall_copy_gbs"] = mall_copy
            rec["roofline"]["frac_vs_mall_copy"] = round(ach / mall_copy, 4)
        out[prec] = rec
        log(f"[bench] 2d {prec} {rec['ms_per_step']:.4f} ms/step")
    out["config"] = {"workload": f"standing_mode_2d m=3 {K}x{K} nu=0.5 kappa=1 waves={list(wl.waves)}",
                     "d": 2, "m": 3, "cells": [K, K], "steps": steps,
                     "adequacy_rule": "nodal error vs exact within 1.1 x the FP64 run's"}
    return out


def run_1d(hl, torch, K=200, m=1):
    """1D m=1 standing wave, 200 cells, nu = 0.5 to T = 1 (400 steps, exact
    U at dt/2), FP64: the whole run through hl_step (graph replay), timed;
    the state against the exact solution at T."""
    from paper_1808_10481_amd import inputs
    wl = inputs.standing_wave_1d(K=K, m=m)
    plan = hl.Plan(1, m, wl.K, dt=wl.dt, c=1.0, precision="fp64")
    p, u = plan.alloc()
    plan.init(p, u, wl.P0, wl.U0)
    plan.step(p, u, wl.steps)                               # warm-up, graph capture
    plan.init(p, u, wl.P0, wl.U0)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record(torch.cuda.current_stream())
    plan.step(p, u, wl.steps)
    e.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    ms = s.elapsed_time(e)
    P, _ = plan.export(p, u)
    ex = wl.exact(wl.steps * wl.dt)
    plan.close()
    return {"us_per_step": 1e3 * ms / wl.steps, "total_ms": ms, "steps": wl.steps,
            "value": K * wl.steps / (ms * 1e-3), "unit": "cell-updates/s",
            "nodal_l2_vs_exact": float(np.sqrt(wl.h[0] * np.sum((P[:, 0] - ex[:, 0]) ** 2))),
            "config": {"workload": f"standing_wave_1d m={m} {K} cells nu=0.5 T=1", "d": 1, "m": m,
                       "cells": [K], "note": "launch-latency bound; hl_step replays 16-step graphs"}}


def run_walls(hl, torch, steps, K=1024, m=3):
    """Walled 2D m=3 1024^2 Gaussian pulse (reflecting boundary, start-up from
    u = 0): `steps` steps timed after 3 untimed ones.  Each step is the ghost
    refresh, the pressure and the velocity half-step."""
    from paper_1808_10481_amd import inputs
    wl = inputs.gaussian_pulse_walls_2d(seed=3, K=K, m=m, steps=steps)
    res, fin = {}, {}
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
        fin[prec] = plan.export(p, u)
        if prec != "fp64":
            res[prec]["rel_l2_vs_fp64_state"] = _rel_state(fin[prec], fin["fp64"])
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
    fin = {}
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
        fin[prec] = plan.export(p, u)
        if prec == "fp64":
            res["fp32"]["rel_l2_vs_fp64_state"] = _rel_state(fin["fp32"], fin["fp64"])
        plan.close()
        del p, u
        torch.cuda.empty_cache()
    res["config"] = {"workload": f"variable_kappa_2d m={m} {K}^2 kappa=1+0.35sin(4pi x)+0.25sin(6pi y), one shot, "
                                 "tuned tile", "d": 2, "m": m, "cells": [K, K]}
    return res


def run_varkappa_3d(hl, torch, steps, K=128, m=2):
    """Variable coefficient in 3D at the headline's order (m=2; one wavefront
    per node): smooth kappa = 1 + 0.35 sin(4 pi x) + 0.25 sin(6 pi y)
    + 0.2 sin(2 pi z) on 128^3 (the kappa Taylor data of 256^3 would take
    29 GB per array in FP64), Gaussian pulse data of width 0.05: `steps` steps
    timed after 2 untimed ones, FP32 and FP64."""
    from paper_1808_10481_amd import inputs
    res = {}
    L = (1.0, 1.0, 1.0)
    amps, waves = (0.35, 0.25, 0.2), (2, 3, 1)
    kp = inputs.kappa_sines(3, m, (K,) * 3, L, amps, waves, "primal")
    ku = inputs.kappa_sines(3, m, (K,) * 3, L, amps, waves, "dual")
    P0 = inputs.gaussian_pulse(3, m, (K,) * 3, L, (0.43, 0.52, 0.61), 0.05)
    fin = {}
    for prec in ("fp32", "fp64"):
        log(f"[bench] variable kappa 3d m={m} {K}^3 {prec}: {steps} steps")
        plan = hl.Plan(3, m, (K,) * 3, cfl=0.5, c=float(np.sqrt(1.8)), precision=prec)
        plan.set_kappa(kp, ku)
        p, u = plan.alloc()
        plan.init(p, u, P0, None)
        plan.step(p, u, 2)
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
        res[prec] = {"value": K ** 3 * steps / (total * 1e-3), "unit": "cell-updates/s",
                     "ms_per_step": total / steps, "p_half_ms": tp, "u_half_ms": tu, "steps": steps}
        fin[prec] = plan.export(p, u)
        if prec == "fp64":
            res["fp32"]["rel_l2_vs_fp64_state"] = _rel_state(fin["fp32"], fin["fp64"])
        plan.close()
        del p, u
        torch.cuda.empty_cache()
    res["config"] = {"workload": f"variable_kappa_3d m={m} {K}^3 kappa=1+0.35sin(4pi x)+0.25sin(6pi y)"
                                 "+0.2sin(2pi z), gaussian pulse width 0.05", "d": 3, "m": m, "cells": [K] * 3}
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
    plans, states, media, cmaxs = [], [], [], []
    nprec = min(2, nshots)
    for K in sizes:
        up = rng.uniform(0.3, 1.0, 2)
        med = inputs.layered_speed(1.0, [up[0], up[1], -(up[0] + up[1])], np.sort(rng.uniform(0.15, 0.85, 3)),
                                   float(rng.uniform(0.02, 0.05)))
        cmax = 1.0 + up[0] + up[1]
        cmaxs.append(cmax)
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
    snap = [(states[i][0].clone(), states[i][1].clone()) for i in range(nprec)]
    ev_s = torch.cuda.Event(enable_timing=True)
    ev_s.record(stream)
    for plan, (p, u) in zip(plans, states):
        plan.step(p, u, steps)
    ev[2].record(stream)
    torch.cuda.synchronize()
    tb, ts = ev[0].elapsed_time(ev[1]) / steps, ev_s.elapsed_time(ev[2]) / steps
    batch.close()
    # precision: the first two shots again in FP64 (same media, sources and
    # step sequence), against their FP32 states after the timed batched steps
    sub = {}
    if nprec > 0:
        plans64, st64 = [], []
        for i in range(nprec):
            K = sizes[i]
            pl = hl.Plan(2, m, (K, K), cfl=0.5, c=float(cmaxs[i]), precision="fp64")
            pl.set_kappa(inputs.kappa_layers(2, m, (K, K), (1.0, 1.0), media[i], "primal"),
                         inputs.kappa_layers(2, m, (K, K), (1.0, 1.0), media[i], "dual"))
            p, u = pl.alloc()
            p.zero_()
            u.zero_()
            plans64.append(pl)
            st64.append((p, u))
        b64 = hl.Batch(plans64)
        b64.set_sources(srcs[:nprec], amps[:nprec])
        # the FP32 shots' sequence: 16 batched steps, 16 per-plan steps, `steps` batched
        b64.step([p for p, _ in st64], [u for _, u in st64], 16)
        for pl, (p, u) in zip(plans64, st64):
            pl.step(p, u, 16)
        b64.step([p for p, _ in st64], [u for _, u in st64], steps)
        torch.cuda.synchronize()
        errs = [_rel_state(plans[i].export(*snap[i]), plans64[i].export(*st64[i])) for i in range(nprec)]
        sub = {"rel_l2_fp32_vs_fp64_state": errs, "shots_compared": nprec}
        b64.close()
        for pl in plans64:
            pl.close()
        del st64
    for plan in plans:
        plan.close()
    del states, ps, us
    torch.cuda.empty_cache()
    return {"batched": {"value": cells / (tb * 1e-3), "unit": "cell-updates/s", "ms_per_step": tb},
            "per_shot": {"value": cells / (ts * 1e-3), "unit": "cell-updates/s", "ms_per_step": ts},
            "speedup_batched_vs_per_shot": ts / tb, "steps": steps, "precision": sub,
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
    res, fin = {}, {}
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
                     "adjoint_cell_updates_per_s": K * K / (adj * 1e-3), "steps": steps,
                     "kappa_gradient": float(g.item())}
        fin[prec] = plan.export(pb, ub)
        if prec == "fp64":
            res["fp32"]["rel_l2_vs_fp64_adjoint_state"] = _rel_state(fin["fp32"], fin["fp64"])
            res["fp32"]["rel_diff_vs_fp64_kappa_gradient"] = abs(res["fp32"]["kappa_gradient"] - float(g.item())) \
                / abs(float(g.item()))
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
    # the same gradient in FP64 (same observed traces), against the FP32 one
    plan64 = hl.Plan(d, m, KK, cfl=0.5, c=cmax, precision="fp64")
    q0, v0 = plan64.alloc()
    plan64.init(q0, v0, inputs.gaussian_pulse(d, m, KK, (1.0, 1.0), centre, 0.05), np.zeros(plan64.host_shapes()[1]))
    kp64 = torch.tensor(km[0], requires_grad=True)
    ku64 = torch.tensor(km[1], requires_grad=True)
    tr64, _, _ = hag.receiver_traces(kp64, ku64, q0, v0, plan64, steps, rec)
    (0.5 * ((tr64.double() - obs) ** 2).sum()).backward()
    g64 = np.concatenate([kp64.grad.numpy().ravel(), ku64.grad.numpy().ravel()])
    g32 = np.concatenate([gp.ravel(), gu.ravel()])
    grad_rel = float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
    plan64.close()
    del q0, v0
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
                         "note": "fourth-order central differences of the FP32 forward"},
            "rel_l2_fp32_vs_fp64_gradient": grad_rel}


def copy_probe(torch, nbytes=1 << 30, reps=20):
    """Plain device copy y <- x of nbytes (the paper's "realistic peak"
    vector-copy measurement); GB/s counts bytes read + written.  1 GiB streams
    from HBM; 64 MiB (128 MiB moved) stays in the 256 MB MALL."""
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
    return {"buffer_bytes": nbytes, "bytes_moved": 2 * nbytes, "avg_ms": round(ms, 4),
            "gbs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


_CPU = {}


def _oracle_sample(job):
    """One CPU worker (single-threaded): the workload's start-up U^{1/2} on the
    dual nodes the sample's pressure half-step reads (untimed), then one
    pressure half-step and one velocity half-step of the oracle over the
    sample nodes S = all x, rows [y0, y0+ny), planes [z0, z0+nz) (timed).
    The velocity half-step reads P^1 on S and the start-up data elsewhere, so
    its result is a true step only on dual nodes whose corners lie in S."""
    import contextlib

    import oracle
    try:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(limits=1)
    except Exception:
        ctx = contextlib.nullcontext()
    wl, prob = _CPU["wl"], _CPU["prob"]
    y0, ny, z0, nz = job
    K = wl.K
    x = np.arange(K[0])

    def nodes(ys, zs):
        g = np.stack(np.meshgrid(x, ys, zs, indexing="ij"), -1).reshape(-1, 3)
        return np.stack([g[:, 0], np.mod(g[:, 1], K[1]), np.mod(g[:, 2], K[2])], -1), g

    with ctx:
        S, loc = nodes(np.arange(y0, y0 + ny), np.arange(z0, z0 + nz))
        dn, _ = nodes(np.arange(y0 - 1, y0 + ny), np.arange(z0 - 1, z0 + nz))
        U = np.zeros((3,) + wl.P0.shape)                   # untouched pages stay unallocated
        uh = oracle.u_half(prob, U, wl.P0, nodes=dn, weight_scale=0.5)
        for i in range(3):
            U[i][tuple(dn.T)] = uh[i]
        t0 = time.perf_counter()
        Pn = oracle.p_half(prob, wl.P0, U, nodes=S)
        P1 = np.zeros_like(wl.P0)
        halo, _ = nodes(np.arange(y0, y0 + ny + 1), np.arange(z0, z0 + nz + 1))
        P1[tuple(halo.T)] = wl.P0[tuple(halo.T)]
        P1[tuple(S.T)] = Pn
        Un = oracle.u_half(prob, U, P1, nodes=S)
        sec = time.perf_counter() - t0
    exact = (loc[:, 1] - y0 + 1 < ny) & (loc[:, 2] - z0 + 1 < nz)
    return dict(seconds=sec, nodes=S, P=Pn, U=Un, exact_u=exact)


def cpu_baseline_3d(wl, workers, ny=32, nz=2):
    """The oracle as it stands, on one step's work over a slab sample of the
    3D workload: `workers` single-threaded processes (fork, before the GPU is
    touched), each on its own block of 256 x ny x nz nodes near the pulse;
    cell-updates/s = sample nodes / the slowest worker's step time.  Then the
    same block once more in this process alone: the 1-core figure."""
    import multiprocessing as mp

    import oracle
    prob = oracle.Problem(3, wl.m, wl.K, wl.length, wl.dt, 1.0)
    _CPU.update(wl=wl, prob=prob)
    K = wl.K[0]
    yc, zc = int(wl.center[1] * K), int(wl.center[2] * K)
    jobs = [((yc - ny // 2) % K, ny, (zc + nz * (w - workers // 2)) % K, nz) for w in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        outs = pool.map(_oracle_sample, jobs)
    wall = time.perf_counter() - t0
    n = sum(len(o["nodes"]) for o in outs)
    slow = max(o["seconds"] for o in outs)
    one = _oracle_sample(jobs[0])
    return {"value": n / slow, "unit": "cell-updates/s", "cores": workers, "kind": "oracle",
            "sample": f"one step's work (the oracle's pressure and velocity half-steps) over {n} nodes: "
                      f"{workers} single-threaded processes, each on {K} x {ny} x {nz} nodes of the "
                      f"{K}^3 grid near the pulse (start-up data computed untimed); slowest worker "
                      f"{slow:.1f} s, pool wall {wall:.1f} s",
            "one_core": {"value": len(one["nodes"]) / one["seconds"], "unit": "cell-updates/s",
                         "seconds": one["seconds"], "nodes": len(one["nodes"])},
            "_outs": outs}


def sample_parity(cb, P1, U1):
    """Relative L2 of the GPU FP64 state after the start-up and one step
    against the oracle's sample: pressure on every sample node, velocity on
    the sample's dual nodes whose corners all lie in the sample."""
    num = den = 0.0
    nu = 0
    for o in cb["_outs"]:
        idx = tuple(o["nodes"].T)
        g = P1[idx]
        num += float(np.sum((g - o["P"]) ** 2))
        den += float(np.sum(o["P"] ** 2))
        sel = o["exact_u"]
        if np.any(sel):
            ii = tuple(o["nodes"][sel].T)
            for i in range(3):
                gu = U1[i][ii]
                num += float(np.sum((gu - o["U"][i][sel]) ** 2))
                den += float(np.sum(o["U"][i][sel] ** 2))
            nu += int(sel.sum())
    return {"rel_l2": float(np.sqrt(num / den)), "p_nodes": int(sum(len(o["nodes"]) for o in cb["_outs"])),
            "u_nodes": nu}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed steps of the 3D headline workload")
    ap.add_argument("--warmup", type=int, default=3, help="untimed steps of the 3D workload after its start-up")
    ap.add_argument("--K", type=int, default=256)
    ap.add_argument("--cpu-workers", type=int, default=0, help="0: the usable cores, at most 16")
    ap.add_argument("--cpu-rows", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-2d", action="store_true")
    ap.add_argument("--steps-2d", type=int, default=1000)
    ap.add_argument("--no-1d", action="store_true")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--no-walls", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-varkappa", action="store_true")
    ap.add_argument("--no-varkappa-3d", action="store_true")
    ap.add_argument("--steps-varkappa-3d", type=int, default=10)
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

    from paper_1808_10481_amd import inputs

    # the CPU baseline forks its workers before anything touches the GPU
    cb = None
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or max(1, min(16, len(os.sched_getaffinity(0))))
        log(f"[bench] cpu baseline: oracle on a slab sample of the 3D workload, {workers} processes")
        wl = inputs.gaussian_pulse_3d(seed=2, K=args.K, m=2, steps=args.steps)
        cb = cpu_baseline_3d(wl, workers, ny=args.cpu_rows)
        del wl
        log(f"[bench] cpu baseline {cb['value']:.3e} cell-updates/s on {cb['cores']} cores "
            f"(1 core {cb['one_core']['value']:.3e})")

    import torch

    from paper_1808_10481_amd import hl
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    probes = {}
    if not args.no_copy_probe:
        probes["hbm"] = copy_probe(torch, 1 << 30)
        probes["mall"] = copy_probe(torch, 64 << 20, reps=200)
        log(f"[bench] copy probes {probes}")

    r3 = run_3d(hl, torch, args.steps, K=args.K, sample=cb, warmup=args.warmup)
    h = r3["fp64"]
    out = {
        "metric": METRIC, "value": h["value"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": h["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": r3["config"]["workload"], "d": 3, "m": 2, "cells": [args.K] * 3,
                   "steps": args.steps, "parallelism": "single_gpu"},
        "roofline": h["roofline"],
        "l2": {"fp64_nodal_rel_l2_vs_exact": h["nodal_rel_l2_vs_exact"],
               "fp64_nodal_l2_vs_exact": h["nodal_l2_vs_exact"]},
        "fp32": r3["fp32"], "fp32_comp": r3["fp32_comp"],
        "gaussian_pulse_3d": {"fp64": h, "config": r3["config"]},
    }
    if "oracle_parity" in r3:
        out["l2"]["fp64_vs_oracle_one_step_sample"] = r3["oracle_parity"]["rel_l2"]
    if cb is not None:
        out["cpu_baseline"] = {k: v for k, v in cb.items() if not k.startswith("_")}
    if probes:
        out["copy_probe"] = probes

    if not args.no_2d:
        out["standing_mode_2d"] = run_2d(hl, torch, args.steps_2d, 20,
                                         mall_copy=probes.get("mall", {}).get("gbs"))
    if not args.no_1d:
        out["standing_wave_1d"] = run_1d(hl, torch)
        log(f"[bench] 1d {out['standing_wave_1d']['us_per_step']:.2f} us/step")
    if not args.no_walls:
        out["gaussian_pulse_walls_2d"] = run_walls(hl, torch, args.steps_walls)
    if not args.no_varkappa:
        out["variable_kappa_2d"] = run_varkappa(hl, torch, args.steps_varkappa)
    if not args.no_varkappa_3d:
        out["variable_kappa_3d"] = run_varkappa_3d(hl, torch, args.steps_varkappa_3d)
    if not args.no_batch:
        out["batched_shots_2d"] = run_batch(hl, torch, args.steps_batch)
    if not args.no_adjoint:
        out["adjoint_2d"] = run_adjoint(hl, torch, args.steps_adjoint)
    if not args.no_kgrad:
        out["kappa_gradient_2d"] = run_kappa_gradient(hl, torch, args.steps_kgrad)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
