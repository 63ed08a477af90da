"""MLBM node-update throughput on one MI355X.

Workload (the Taylor-Green configuration at full size): a 512 x 512 lattice on
[0, 2 pi)^2 with every coordinate jittered by U[-0.3 h, 0.3 h] (seed 2),
N = 262,144 nodes, D2Q9 BGK, tau = 0.6, u0 = 0.01, streaming distance dx = h,
r^3 RBF with degree-4 polynomial augmentation on K = 30 stencils, the paper's
stencil rule (closest node of each departure point), FP32 deviation-stored
populations. A timed step is one fused stream+collide pass over all nodes;
the weight build is timed separately.

Also reported: the same step in plain FP64, the adjoint/forward cost of a
checkpointed reverse sweep and of one reversed step, L2 errors against the
analytic decay, the roofline position of the step kernel, the weight-build
rate, the annular channel (about 490,000 Poisson-disk nodes with walls and
body force), 64 uneven clouds in one graph, and the FP64 CPU oracle run on the
benchmarked cloud itself: the velocity of the timed FP32 and FP64 states and
of the 2,000-step states against the oracle's, node by node, and the oracle's
own rate on the host cores.

Timing: the K timed steps are one HIP graph replayed 5 times; ms_per_step is
the median replay over K (min and max are reported beside it).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLBM node-updates/s FP32 vs FP64 + adjoint/forward cost, at stated L2 vs oracle"
HBM_PEAK_GBS = 8000.0
PROFILE_PMC = os.path.join(ROOT, "profiles", "step_fp32_tgv512_pmc.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


L2_STEPS = 2000   # length of the Taylor-Green run at which accuracy is reported


def bytes_per_update(K: int, precision: str, paper_mode: bool) -> int:
    """Algorithmic HBM bytes of one node-update: 8K weights, K stencil
    indices, 9 populations read and 9 written (gathers counted once), plus 8
    owner indices with the paper's stencil rule."""
    if precision == "f32":
        b = 4 * (8 * K + K + 9 + 9)
    else:
        b = 8 * 8 * K + 4 * K + 8 * 18
    return b + (32 if paper_mode else 0)


def adjoint_bytes_per_update(K: int) -> float:
    """What one reversed FP32 step must move per node with the tile-local
    transposed operator: 8K entries of (4-byte weight + 10-bit position),
    8 row pointers, f^n (36 B), lambda^{n+1} once (36 B), lambda^n (36 B)."""
    return 8 * K * (4 + 4 / 3) + 8 * 4 + 3 * 36


def step_kernel_name(variant: int) -> str:
    """The FP32 step kernel of the headline configuration (paper stencils, no
    force, no walls) that an autotuner variant launches, as a kernel trace
    names it."""
    nt = "true" if variant % 2 else "false"
    if 6 <= variant <= 9:
        return "k_step32s<0, false, 0, false, %s, %d>" % (nt, 2 if variant >= 8 else 1)
    if 0 <= variant <= 5:
        return "k_step32<0, false, 0, false, %d, %s>" % (1 + variant // 2, nt)
    return "k_step32<0, false, 0, false, 1, false>"


def step_kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("step.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_2306_01525_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TIMING_REPS = 5   # replays of the timed graph; the median is reported
BUILD_REPS = 3    # warm weight builds; the median is reported


def time_steps(plan, g, steps, warmup, stream, reps=TIMING_REPS):
    """W eager warm-up steps, then a HIP graph of K steps replayed `reps` times,
    each replay bracketed by synchronisation and timed with events on the
    launch stream. Returns the per-replay milliseconds (in replay order), the
    final state and the number of steps taken from g. With K even every replay
    continues from the last one; with K odd each replay repeats the same K
    steps from the same input."""
    import torch
    other = plan.new_state()
    times = []
    with torch.cuda.stream(stream):
        res = plan.step(g, other, warmup, stream=stream)
        if res is other:
            g, other = other, g
        plan.graph_create(g, other, steps, stream)
        torch.cuda.synchronize()
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            plan.graph_launch(stream)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
    final = other if steps % 2 else g
    taken = warmup + (steps if steps % 2 else steps * reps)
    return times, final, taken


def timing_summary(times, steps):
    """Median, min and max of the per-replay times, per step."""
    t = sorted(times)
    return {"replays": len(t), "steps_per_replay": steps,
            "ms_per_step_median": t[len(t) // 2] / steps, "ms_per_step_min": t[0] / steps,
            "ms_per_step_max": t[-1] / steps}


def run_gpu(args):
    import numpy as np
    import torch
    from paper_2306_01525_amd import MLBM_FP32_DEV, MLBM_FP64, Params, Plan
    from paper_2306_01525_amd import targets
    from paper_2306_01525_amd.autograd import Rollout
    from synth import jittered_lattice, tgv_initial_velocity

    n_side, K, m, tau, u0, seed = 512, 30, 4, 0.6, 0.01, 2
    c = jittered_lattice(n_side, seed=seed)
    L = c.period[0]
    ux, uy = tgv_initial_velocity(c.x, c.y, L, u0)
    dev = torch.device("cuda:0")
    xt = torch.tensor(c.x, device=dev)
    yt = torch.tensor(c.y, device=dev)
    uxt = torch.tensor(ux, device=dev)
    uyt = torch.tensor(uy, device=dev)
    stream = torch.cuda.Stream()
    out = {}

    def build(precision, with_adjoint=0):
        p = Params(dx=c.h, K=K, degree=m, tau=tau, stencil_mode=0, precision=precision,
                   with_adjoint=with_adjoint)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = Plan.build(xt, yt, c.period, p, stream=stream)
        torch.cuda.synchronize()
        return plan, (time.perf_counter() - t0) * 1e3

    # FP32 deviation form: the headline. The first build of the process also
    # pays one-time costs (code objects, library set-up); the build time
    # reported is the median of the three builds after it.
    log("building FP32 plan, N =", c.n)
    plan32, build_cold_ms = build(MLBM_FP32_DEV)
    build_warm = []
    for _ in range(BUILD_REPS):
        plan32.close()
        plan32, t = build(MLBM_FP32_DEV)
        build_warm.append(t)
    build_ms = float(np.median(build_warm))
    a, b = plan32.new_state(), plan32.new_state()
    tune_ms = plan32.autotune(plan32.init(uxt, uyt, g=a), b, 20)
    out["tune"] = {"ms_per_step": tune_ms, "chosen": int(plan32.info.variant)}
    log("autotune ms/step per variant:", " ".join("%.4f" % m for m in tune_ms),
        "-> variant", plan32.info.variant)
    del a, b
    log("build %.1f ms; timing %d FP32 steps after %d warm-up, %d replays"
        % (build_ms, args.steps, args.warmup, TIMING_REPS))
    g = plan32.init(uxt, uyt)
    torch.cuda.synchronize()
    t32, g32, taken = time_steps(plan32, g, args.steps, args.warmup, stream)
    out["timing32"] = timing_summary(t32, args.steps)
    ms32 = out["timing32"]["ms_per_step_median"] * args.steps
    # velocity of the timed state (kept for the comparison with the oracle),
    # then the state is stepped on to the workload's full length (2,000 steps)
    fields = {"fp32": {}, "fp64": {}}
    _, u, v = plan32.moments(g32)
    fields["fp32"][taken] = (u.cpu().numpy(), v.cpu().numpy())
    total = max(L2_STEPS, taken)
    g32 = plan32.step(g32, plan32.new_state(), total - taken)
    tx, ty = targets.tgv_velocity(c.x, c.y, L, u0, tau, c.h, total)
    tx_t, ty_t = torch.tensor(tx, device=dev), torch.tensor(ty, device=dev)
    l2u32, l2v32 = plan32.l2(g32, tx_t, ty_t)
    _, u32, v32 = plan32.moments(g32)
    fields["fp32"][total] = (u32.cpu().numpy(), v32.cpu().numpy())
    out.update(ms32=ms32, build_ms=build_ms, build_cold_ms=build_cold_ms,
               build_warm_ms=build_warm, l2_32=(l2u32, l2v32),
               l2_steps=total, timed_state_steps=taken, fields=fields, cloud=c,
               velocity0=(ux, uy), tau=tau, degree=m)
    log("FP32: %.4f ms/step (median of %d replays; min %.4f, max %.4f), L2(u) vs analytic %.3e"
        % (ms32 / args.steps, TIMING_REPS, out["timing32"]["ms_per_step_min"],
           out["timing32"]["ms_per_step_max"], l2u32))

    # The step's data (310 MB) is close to the 256 MB Infinity Cache, so part
    # of it is still cached from the previous step. A second plan of the same
    # cloud stepped in between doubles the working set: that rate is the one
    # with every byte from HBM.
    planB, _ = build(MLBM_FP32_DEV)
    planB.set_variant(int(plan32.info.variant))
    pair = [[plan32, plan32.init(uxt, uyt), plan32.new_state()],
            [planB, planB.init(uxt, uyt), planB.new_state()]]

    def interleaved(n):
        with torch.cuda.stream(stream):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(n):
                for q in pair:
                    q[0].step(q[1], q[2], 1, stream=stream)
                    q[1], q[2] = q[2], q[1]
            e1.record(stream)
            torch.cuda.synchronize()
        return e0.elapsed_time(e1) / (2 * n)

    # 20 steps of each plan per replay: enough for a stable median, and few
    # enough that these slower launches of the headline kernel stay a small
    # share of its dispatches in a kernel trace of the default run
    cold_steps = min(args.steps, 20)
    interleaved(10)
    ms_cold = sorted(interleaved(cold_steps) for _ in range(TIMING_REPS))[TIMING_REPS // 2]
    out["ms_cold"] = ms_cold
    log("FP32 with a second plan stepped in between (twice the working set): %.4f ms/step"
        % ms_cold)
    planB.close()
    del pair
    out["copy_bw"] = copy_bandwidth()
    log("torch device copy of 1 GiB: %.0f GB/s" % out["copy_bw"]["achieved"])

    # FP64 plain form, same number of steps
    if not args.skip_fp64:
        plan64, build64_ms = build(MLBM_FP64)
        g = plan64.init(uxt, uyt)
        t64, g64, taken64 = time_steps(plan64, g, args.steps, args.warmup, stream)
        out["timing64"] = timing_summary(t64, args.steps)
        ms64 = out["timing64"]["ms_per_step_median"] * args.steps
        _, u, v = plan64.moments(g64)
        fields["fp64"][taken64] = (u.cpu().numpy(), v.cpu().numpy())
        g64 = plan64.step(g64, plan64.new_state(), total - taken64)
        l2u64, l2v64 = plan64.l2(g64, tx_t, ty_t)
        _, u64, v64 = plan64.moments(g64)
        fields["fp64"][total] = (u64.cpu().numpy(), v64.cpu().numpy())
        d = torch.sqrt(((u32 - u64) ** 2 + (v32 - v64) ** 2).sum() / (u64 ** 2 + v64 ** 2).sum())
        out.update(ms64=ms64, l2_64=(l2u64, l2v64), fp32_vs_fp64=float(d))
        log("FP64: %.4f ms/step, L2(u) vs analytic %.3e, FP32 vs FP64 %.3e"
            % (ms64 / args.steps, l2u64, float(d)))
        plan64.close()
        del plan64

    # adjoint / forward cost: one segment of C steps forward vs recompute + reverse
    if not args.skip_adjoint:
        C = 50
        planA, _ = build(MLBM_FP32_DEV, with_adjoint=1)
        planA.set_variant(plan32.info.variant)
        with torch.cuda.stream(stream):
            ro = Rollout(planA, C, C)
            ro.forward(uxt, uyt, stream=stream)      # warm
            ro.loss(tx_t, ty_t, stream=stream)
            ro.backward(stream=stream)
            torch.cuda.synchronize()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e0, e1 = e[0], e[2]
            e[0].record(stream)
            ro.forward(uxt, uyt, stream=stream)
            ro.loss(tx_t, ty_t, stream=stream)
            e[1].record(stream)
            ro.backward(stream=stream)
            e[2].record(stream)
            torch.cuda.synchronize()
        fwd = e[0].elapsed_time(e[1])
        bwd = e[1].elapsed_time(e[2])
        out.update(adj_ratio=bwd / fwd, adj_fwd_ms=fwd, adj_bwd_ms=bwd)
        log("adjoint: forward %.2f ms, recompute+reverse %.2f ms, ratio %.2f" % (fwd, bwd, bwd / fwd))
        # one reversed step on its own (gather + collision VJP + d/dtau partials)
        with torch.cuda.stream(stream):
            fn = planA.init(uxt, uyt)
            lam_a = torch.randn_like(fn)
            lam_b = torch.empty_like(fn)
            dtau = torch.zeros(1, dtype=torch.float64, device=dev)
            reps = 50
            for _ in range(5):
                planA.step_adjoint(fn, lam_a, lam_b, dtau, stream=stream)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                planA.step_adjoint(fn, lam_a, lam_b, dtau, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
        out["adj_step_ms"] = e0.elapsed_time(e1) / reps
        log("adjoint step alone: %.4f ms" % out["adj_step_ms"])
        # the whole adjoint workload: 500 steps checkpointed every 50
        # (forward with checkpoints + loss, then recompute + reverse sweep)
        T = 500
        with torch.cuda.stream(stream):
            del fn, lam_a, lam_b
            torch.cuda.synchronize()
            torch.cuda.reset_peak_memory_stats()
            base_mem = torch.cuda.memory_allocated()
            ro = Rollout(planA, T, C)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream)
            ro.forward(uxt, uyt, stream=stream)
            ro.loss(tx_t, ty_t, stream=stream)
            e[1].record(stream)
            ro.backward(stream=stream)
            e[2].record(stream)
            torch.cuda.synchronize()
        out["rollout"] = {"steps": T, "segment": C, "forward_loss_ms": e[0].elapsed_time(e[1]),
                          "backward_ms": e[1].elapsed_time(e[2]),
                          "ratio": e[1].elapsed_time(e[2]) / e[0].elapsed_time(e[1]),
                          "peak_extra_bytes": torch.cuda.max_memory_allocated() - base_mem,
                          "plan_bytes": int(planA._buf.numel())}
        log("rollout of %d steps: forward+loss %.1f ms, backward %.1f ms, peak extra memory "
            "%.2f GB" % (T, out["rollout"]["forward_loss_ms"], out["rollout"]["backward_ms"],
                          out["rollout"]["peak_extra_bytes"] / 1e9))
        del ro
        # the same 500 steps with every pre-collision state kept by the
        # forward (T + 1 states, 4.7 GB): the backward is the reversed steps
        # alone. One untimed run first, so that the timed one reuses the
        # allocator's blocks.
        with torch.cuda.stream(stream):
            for timed in (False, True):
                torch.cuda.synchronize()
                torch.cuda.reset_peak_memory_stats()
                base_mem = torch.cuda.memory_allocated()
                ro = Rollout(planA, T, C, store_all=True)
                e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                e[0].record(stream)
                ro.forward(uxt, uyt, stream=stream)
                ro.loss(tx_t, ty_t, stream=stream)
                e[1].record(stream)
                ro.backward(stream=stream)
                e[2].record(stream)
                torch.cuda.synchronize()
                peak = torch.cuda.max_memory_allocated() - base_mem
                del ro
        out["rollout_stored"] = {"steps": T, "forward_loss_ms": e[0].elapsed_time(e[1]),
                                 "backward_ms": e[1].elapsed_time(e[2]),
                                 "ratio": e[1].elapsed_time(e[2]) / e[0].elapsed_time(e[1]),
                                 "peak_extra_bytes": peak}
        log("rollout of %d steps, every state stored: forward+loss %.1f ms, backward %.1f ms, "
            "peak extra memory %.2f GB" % (T, out["rollout_stored"]["forward_loss_ms"],
                                           out["rollout_stored"]["backward_ms"], peak / 1e9))
        planA.close()
    out["n"] = c.n
    out["K"] = K
    plan32.close()
    return out


def run_tgv40():
    """The small Taylor-Green workload: 40 x 40 jittered lattice (seed 1),
    1,600 nodes, K = 12, degree 2, own-node stencils (the paper's rule
    diverges at K = 12 with degree 2 on these clouds), tau = 0.8, u0 = 0.01,
    200 steps; FP32 and FP64 steps timed as for the headline, L2 against the
    analytic decay and against the oracle after the 200 steps, and the oracle's
    own rate on the host (all threads and one). The whole cloud sits in L2, so
    this is a latency figure, not a roofline point."""
    import numpy as np
    import torch
    import oracle
    from paper_2306_01525_amd import MLBM_FP32_DEV, MLBM_FP64, MLBM_STENCIL_OWN, Params, Plan
    from paper_2306_01525_amd import targets
    from synth import jittered_lattice, tgv_initial_velocity
    steps, K, m, tau, u0 = 200, 12, 2, 0.8, 0.01
    c = jittered_lattice(40, seed=1)
    ux, uy = tgv_initial_velocity(c.x, c.y, c.period[0], u0)
    tx, ty = targets.tgv_velocity(c.x, c.y, c.period[0], u0, tau, c.h, steps)
    nbr, own, W = oracle.build_plan(c, c.h, K, m, mode=1)
    f0 = oracle.equilibrium(np.ones(c.n), ux, uy)
    threads = oracle.threads()
    t0 = time.perf_counter()
    f = oracle.run(f0, nbr, own, W, tau, steps)
    t_all = time.perf_counter() - t0
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.run(f0, nbr, own, W, tau, steps)
    t_one = time.perf_counter() - t0
    oracle.set_threads(threads)
    _, uo, vo = oracle.moments(f)
    out = {"nodes": c.n, "K": K, "degree": m, "tau": tau, "steps": steps, "stencil": "own",
           "oracle": {"value_all_threads": c.n * steps / t_all, "threads": threads,
                      "value_one_thread": c.n * steps / t_one}}
    stream = torch.cuda.Stream()
    for prec, name in ((MLBM_FP32_DEV, "fp32"), (MLBM_FP64, "fp64")):
        p = Params(dx=c.h, K=K, degree=m, tau=tau, stencil_mode=MLBM_STENCIL_OWN, precision=prec)
        plan = Plan.build(c.x, c.y, c.period, p)
        times, _, _ = time_steps(plan, plan.init(ux, uy), steps, 0, stream)
        g = plan.step(plan.init(ux, uy), plan.new_state(), steps)
        _, u, v = (a.cpu().numpy() for a in plan.moments(g))
        t = timing_summary(times, steps)
        out[name] = {"ms_per_step": t["ms_per_step_median"], "timing": t,
                     "value": c.n / (t["ms_per_step_median"] / 1e3),
                     "l2_vs_analytic_u": float(np.linalg.norm(u - tx) / np.linalg.norm(tx)),
                     "l2_vs_oracle": field_error(u, v, uo, vo)}
        plan.close()
    log("TGV-40: FP32 %.4f ms/step, L2 vs oracle %.2e; FP64 %.4f ms/step"
        % (out["fp32"]["ms_per_step"], out["fp32"]["l2_vs_oracle"]["rel_l2"],
           out["fp64"]["ms_per_step"]))
    return out


def run_annulus(steps: int, warmup: int):
    """The annular channel at about 490,000 Poisson-disk nodes (R1 = 1, R2 = 2,
    seed 3): K = 20, degree 3, paper stencils, dx = h, tau = 0.7, equilibrium
    walls, azimuthal force of the paper's flow (g = 1e-6 at dx_ML = 1/160
    carried to dx = h under diffusive scaling). FP32 steps timed as for the
    headline."""
    import numpy as np
    import torch
    from paper_2306_01525_amd import Params, Plan
    from synth.clouds import annulus_force, annulus_h_for_count, annulus_poisson
    c = annulus_poisson(1.0, 2.0, annulus_h_for_count(1.0, 2.0, 500_000), seed=3)
    K = 20
    p = Params(dx=c.h, K=K, degree=3, tau=0.7, stencil_mode=0, force_kind=1,
               force_mag=annulus_force(c.h), wall_kind=1, rho_wall=1.0)
    log("annulus: n = %d, h = %.3e; building" % (c.n, c.h))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = Plan.build(c.x, c.y, c.period, p, node_type=c.node_type)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    stream = torch.cuda.Stream()
    zeros = np.zeros(c.n)
    tune = plan.autotune(plan.init(zeros, zeros), plan.new_state(), 20)
    log("annulus: autotune ms/step per variant:", " ".join("%.4f" % t for t in tune),
        "-> variant", plan.info.variant)
    times, g, _ = time_steps(plan, plan.init(zeros, zeros), steps, warmup, stream)
    timing = timing_summary(times, steps)
    _, u, v = plan.moments(g)
    bpu = bytes_per_update(K, "f32", True)
    per = timing["ms_per_step_median"]
    out = {"nodes": c.n, "K": K, "degree": 3, "steps": steps, "ms_per_step": per,
           "value": c.n / (per / 1e3), "bytes_per_update": bpu, "timing": timing,
           "roofline_frac": bpu * c.n / (per / 1e3) / 1e9 / HBM_PEAK_GBS,
           "build_ms": build_ms, "fallback_tiles": int(plan.info.fallback_tiles),
           "autotune_ms_per_step": tune, "variant": int(plan.info.variant),
           "max_speed": float(torch.sqrt(u * u + v * v).max()),
           "device_error": plan.device_error()}
    log("annulus: %.4f ms/step, %.2e node-updates/s" % (per, out["value"]))
    plan.close()
    return out


def run_lbm(steps: int, warmup: int, l2_steps: int, ml_l2: float, ml_ms: float):
    """The paper's reference method, standard LBM with index-shift streaming,
    on the regular 512 x 512 lattice of the same Taylor-Green flow (equal
    node count to the MLBM cloud): L2 against the analytic decay after the same
    steps, and the step time (HIP graph of the steps, as for the MLBM); then a
    2048 x 2048 lattice for the bandwidth figure (72 B per node-update)."""
    import numpy as np
    import torch
    from paper_2306_01525_amd import targets
    from paper_2306_01525_amd.lbm import Lattice
    tau, u0 = 0.6, 0.01
    out = {}
    for side in (512, 2048):
        lat = Lattice(side, side, tau)
        ix, iy = np.meshgrid(np.arange(side), np.arange(side))
        x, y = ix.ravel().astype(float), iy.ravel().astype(float)
        k = 2 * math.pi / side
        ux, uy = u0 * np.sin(k * x) * np.cos(k * y), -u0 * np.cos(k * x) * np.sin(k * y)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            g = lat.init(ux, uy, stream=stream)
            other = lat.new_state()
            res = lat.step(g, other, warmup, stream=stream)
            if res is other:
                g, other = other, g
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream):
                lat.step(g, other, steps, stream=stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            graph.replay()
            e1.record(stream)
            torch.cuda.synchronize()
        final = other if steps % 2 else g
        per = e0.elapsed_time(e1) / steps
        final = lat.step(final, g if final is other else other, l2_steps - steps - warmup)
        _, u, v = lat.moments(final)
        tx, _ = targets.tgv_velocity(x, y, float(side), u0, tau, 1.0, l2_steps)
        ug = u.cpu().numpy()
        l2 = float(np.linalg.norm(ug - tx) / np.linalg.norm(tx))
        ach = 72.0 * lat.n / (per / 1e3) / 1e9
        out["%dx%d" % (side, side)] = {"ms_per_step": per, "value": lat.n / (per / 1e3),
                                         "roofline_frac": ach / HBM_PEAK_GBS, "l2_vs_analytic_u": l2}
        log("LBM %dx%d: %.4f ms/step, %.2e node-updates/s, L2(u) %.3e"
            % (side, side, per, lat.n / (per / 1e3), l2))
        del graph, g, other
    eq = out["512x512"]
    out["mlbm_over_lbm_equal_n"] = {"l2_ratio": ml_l2 / eq["l2_vs_analytic_u"],
                                   "time_ratio": ml_ms / eq["ms_per_step"]}
    return out


def run_batched(steps: int):
    """64 Taylor-Green clouds of uneven size (10^4 to 2x10^5 nodes,
    log-uniform, seed 4), each with its own tau in [0.55, 1] and degree 2-4
    (K 20/25/30), the paper's stencil rule, FP32. One HIP graph holds the
    weight build of all clouds, the initial state and `steps` steps; it is
    launched once and timed, and the steps alone are timed from a second
    graph."""
    import numpy as np
    import torch
    from paper_2306_01525_amd import MLBM_STENCIL_PAPER, Params, Plan
    from synth import batched_tgv_specs, jittered_lattice, tgv_initial_velocity
    specs = batched_tgv_specs(64, seed=4)
    clouds, params, ux, uy = [], [], [], []
    for sp in specs:
        c = jittered_lattice(sp["n_side"], seed=sp["seed"])
        a, b = tgv_initial_velocity(c.x, c.y, c.period[0], 0.01)
        clouds.append((c.x, c.y, c.period, None))
        params.append(Params(dx=c.h, K=sp["K"], degree=sp["degree"], tau=sp["tau"],
                             stencil_mode=MLBM_STENCIL_PAPER))
        ux.append(a)
        uy.append(b)
    ux, uy = np.concatenate(ux), np.concatenate(uy)
    n_total = ux.shape[0]
    log("batched: %d clouds, %d nodes; eager build + autotune" % (len(clouds), n_total))
    eager = Plan.build_batch(clouds, params)
    a, b = eager.new_state(), eager.new_state()
    tune = eager.autotune(eager.init(ux, uy, g=a), b, 10)
    variant = int(eager.info.variant)
    del a, b
    stream = torch.cuda.Stream()
    # steps only
    with torch.cuda.stream(stream):
        g0 = eager.init(ux, uy, stream=stream)
        g1 = eager.new_state()
        eager.graph_create(g0, g1, steps, stream)
        eager.graph_launch(stream)                     # warm
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        eager.graph_launch(stream)
        e1.record(stream)
        torch.cuda.synchronize()
    steps_ms = e0.elapsed_time(e1)
    eager.close()
    # build + init + steps in one graph
    plan, g_a, g_b, res = Plan.build_graph(clouds, params, ux, uy, steps, stream, variant)
    plan.graph_launch(stream)                          # warm
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    plan.graph_launch(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    full_ms = e0.elapsed_time(e1)
    err = plan.device_error()
    # the same steps on the plan that graph built: its tile LDS was sized at
    # capture time (the capacity bound, the halo sizes being unknown until
    # the build has run), so its steps can be slower than the eager plan's;
    # the build + init share of the one-graph run is the difference
    with torch.cuda.stream(stream):
        plan.graph_create(res, g_a if res is g_b else g_b, steps, stream)
        plan.graph_launch(stream)                      # warm
        torch.cuda.synchronize()
        e0.record(stream)
        plan.graph_launch(stream)
        e1.record(stream)
        torch.cuda.synchronize()
    steps_cap_ms = e0.elapsed_time(e1)
    plan.close()
    log("batched: build+init+%d steps %.1f ms in one graph; steps alone %.1f ms (eager plan), "
        "%.1f ms (the graph's plan)" % (steps, full_ms, steps_ms, steps_cap_ms))
    return {"clouds": len(clouds), "nodes": int(n_total), "steps": steps,
            "graph_ms_build_init_steps": full_ms, "graph_ms_steps": steps_ms,
            "graph_ms_steps_capture_sized_plan": steps_cap_ms,
            "build_init_ms": full_ms - steps_cap_ms,
            "node_updates_per_s_steps": n_total * steps / (steps_ms / 1e3),
            "node_updates_per_s_incl_build": n_total * steps / (full_ms / 1e3),
            "variant": variant, "autotune_ms_per_step": tune, "device_error": err}


def field_error(u, v, uo, vo):
    """Relative L2 of the velocity against the oracle's, and the largest
    per-node error |u - u_o| over the largest oracle speed."""
    import numpy as np
    du = np.hypot(u - uo, v - vo)
    return {"rel_l2": float(np.sqrt((du ** 2).sum() / (uo ** 2 + vo ** 2).sum())),
            "max_node_rel": float(du.max() / np.hypot(uo, vo).max())}


def oracle_leg(r):
    """The FP64 CPU oracle on the benchmarked cloud itself (the 262,144-node
    Taylor-Green cloud, same K, degree, tau and stencil rule): its stencils,
    owners (k-d tree candidates, exact selection) and shape vectors, then the
    time loop to every step count at which the GPU states were kept. Returns
    the error of each GPU state against the oracle's and the oracle's own
    rates: all host threads over the whole run, and one thread over 3 steps."""
    import numpy as np
    import oracle
    c = r["cloud"]
    ux, uy = r["velocity0"]
    tau, K, m = r["tau"], r["K"], r["degree"]
    threads = oracle.threads()
    t0 = time.perf_counter()
    nbr, own, W = oracle.build_plan(c, c.h, K, m, mode=0, search="tree")
    build_s = time.perf_counter() - t0
    log("oracle: built stencils, owners and shape vectors in %.1f s on %d threads"
        % (build_s, threads))
    f = oracle.equilibrium(np.ones(c.n), ux, uy)
    marks = sorted({s for flds in r["fields"].values() for s in flds})
    errs = {prec: {} for prec in r["fields"]}
    done, step_s = 0, 0.0
    for s in marks:
        t0 = time.perf_counter()
        f = oracle.run(f, nbr, own, W, tau, s - done)
        step_s += time.perf_counter() - t0
        done = s
        _, uo, vo = oracle.moments(f)
        for prec, flds in r["fields"].items():
            if s in flds:
                errs[prec][str(s)] = field_error(flds[s][0], flds[s][1], uo, vo)
        log("oracle: step %d after %.1f s; " % (s, step_s) +
            ", ".join("%s rel L2 %.3e, max node %.3e" % (p, e[str(s)]["rel_l2"],
                                                         e[str(s)]["max_node_rel"])
                      for p, e in errs.items() if str(s) in e))
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.run(f, nbr, own, W, tau, 3)
    one_s = time.perf_counter() - t0
    oracle.set_threads(threads)
    # one segment of the adjoint workload: 50 steps forward (kept), then 50
    # reversed steps of the discrete adjoint, on all threads
    from paper_2306_01525_amd import targets
    seg = 50
    tx, ty = targets.tgv_velocity(c.x, c.y, c.period[0], 0.01, tau, c.h, seg)
    t0 = time.perf_counter()
    oracle.adjoint(nbr, own, W, tau, seg, 1.0, ux, uy, tx, ty)
    adj_s = time.perf_counter() - t0
    fwd_s = step_s / done * seg
    log("oracle: %d forward + %d reversed steps in %.2f s (forward alone %.2f s)"
        % (seg, seg, adj_s, fwd_s))
    base = {"value": c.n * done / step_s, "unit": "node-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "FP64 oracle on the benchmarked TGV-512 cloud itself (262,144 nodes, K 30, "
                      "degree 4, tau 0.6, paper stencils): %d steps in %.1f s on %d threads after "
                      "a %.1f s build of stencils, owners and shape vectors"
                      % (done, step_s, threads, build_s),
            "build_s": build_s, "one_thread_value": c.n * 3 / one_s,
            "adjoint_segment": {"steps": seg, "forward_and_reverse_s": adj_s,
                                "forward_s": fwd_s,
                                "reverse_over_forward": (adj_s - fwd_s) / fwd_s},
            "search_fallbacks": dict(oracle.last_fallbacks)}
    return errs, base


COPY_BYTES = 256 << 20


def copy_bandwidth(reps=5):
    """HBM bandwidth of torch's device copy of 1 GiB (read and write), the
    median of `reps` copies: a plain streaming kernel beside the roofline."""
    import torch
    x = torch.ones((1 << 30) // 4, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = sorted(ts)[reps // 2]
    del x, y
    return {"bytes": 2 << 30, "ms": ms, "achieved": (2 << 30) / (ms * 1e-3) / 1e9, "unit": "GB/s"}


def copy_calibration():
    """A plain elementwise copy of known size (reads and writes COPY_BYTES)
    for scaling the HBM byte counters."""
    import torch
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()


def _read_counter_csv(path):
    import csv
    rows = []
    for root, _, files in os.walk(path):
        for f in files:
            if f.endswith("counter_collection.csv"):
                with open(os.path.join(root, f)) as fh:
                    rows.extend(csv.DictReader(fh))
    return rows


def summarize_pmc(fetch_dir, write_dir, command):
    """Per-dispatch FETCH_SIZE and WRITE_SIZE (KiB) of the step kernel and of
    the copy kernel, the copy-based scale factor, and the HBM bytes per step
    launch; writes the JSON that bench.py reads and prints a text summary."""
    def per_kernel(rows, counter):
        acc = {}
        for r in rows:
            name = r.get("Kernel_Name", "")
            if r.get("Counter_Name", "") != counter:
                continue
            acc.setdefault(name, {})
            did = r.get("Dispatch_Id", str(len(acc[name])))
            acc[name][did] = acc[name].get(did, 0.0) + float(r["Counter_Value"])
        return {k: sorted(v.values()) for k, v in acc.items()}

    fetch = per_kernel(_read_counter_csv(fetch_dir), "FETCH_SIZE")
    write = per_kernel(_read_counter_csv(write_dir), "WRITE_SIZE")
    # the headline kernel: the TGV step (paper stencils, no force, no walls,
    # no recording) in whichever variant the autotuner kept
    steps = [k for k in fetch if ("k_step32s<0, false, 0, false" in k or
                                  "k_step32<0, false, 0, false" in k)]
    step = max(steps, key=lambda k: len(fetch[k]))
    copy = [k for k in fetch if "elementwise" in k and "mul" in k.lower()]
    copy = max(copy, key=lambda k: len(fetch[k]))

    def median(v):
        return v[len(v) // 2]

    fk_copy, wk_copy = median(fetch[copy]), median(write[copy])
    f_scale = (COPY_BYTES / 1024.0) / fk_copy
    w_scale = (COPY_BYTES / 1024.0) / wk_copy
    fk, wk = median(fetch[step]), median(write[step])
    bytes_launch = fk * 1024.0 * f_scale + wk * 1024.0 * w_scale
    out = {"kernel": step, "kernel_hash": step_kernel_hash(), "dispatches": len(fetch[step]),
           "fetch_kib": fk, "write_kib": wk, "copy_kernel": copy, "copy_fetch_kib": fk_copy,
           "copy_write_kib": wk_copy, "copy_bytes": COPY_BYTES, "fetch_scale": f_scale,
           "write_scale": w_scale, "bytes_per_launch": bytes_launch, "command": command}
    os.makedirs(os.path.dirname(PROFILE_PMC), exist_ok=True)
    with open(PROFILE_PMC, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def summarize_traffic(fetch_dir, write_dir, out_path, command):
    """Per-dispatch HBM bytes of every kernel seen in two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE), scaled by the same counters read on the copy
    kernel of known size (run with --copy-calibration); written as a text
    table of every kernel, largest first."""
    def per_kernel(rows, counter):
        acc = {}
        for r in rows:
            if r.get("Counter_Name", "") != counter:
                continue
            name = r.get("Kernel_Name", "")
            did = r.get("Dispatch_Id", str(len(acc.get(name, {}))))
            acc.setdefault(name, {})
            acc[name][did] = acc[name].get(did, 0.0) + float(r["Counter_Value"])
        return {k: sorted(v.values()) for k, v in acc.items()}

    fetch = per_kernel(_read_counter_csv(fetch_dir), "FETCH_SIZE")
    write = per_kernel(_read_counter_csv(write_dir), "WRITE_SIZE")
    copy = max((k for k in fetch if "elementwise" in k and "mul" in k.lower()),
               key=lambda k: len(fetch[k]))
    med = lambda v: v[len(v) // 2]
    f_scale = (COPY_BYTES / 1024.0) / med(fetch[copy])
    w_scale = (COPY_BYTES / 1024.0) / med(write[copy])
    rows = []
    for k in fetch:
        if k not in write or "elementwise" in k:
            continue
        fb, wb = med(fetch[k]) * 1024.0 * f_scale, med(write[k]) * 1024.0 * w_scale
        rows.append((fb + wb, len(fetch[k]), fb, wb, k))
    rows.sort(reverse=True)
    lines = ["# HBM bytes per dispatch (median over dispatches) from rocprofv3 FETCH_SIZE and",
             "# WRITE_SIZE, scaled by the copy kernel of %d bytes: FETCH x %.4f, WRITE x %.4f"
             % (COPY_BYTES, f_scale, w_scale),
             "# command: " + command,
             "%-10s %12s %12s %12s  %s" % ("dispatches", "fetch_MB", "write_MB", "total_MB", "kernel")]
    for tot, nd, fb, wb, k in rows:
        lines.append("%-10d %12.1f %12.1f %12.1f  %s" % (nd, fb / 1e6, wb / 1e6, tot / 1e6, k[:110]))
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_sq(dirs, kernels, out_path, command):
    """Per-wavefront SQ counters (sum over the dispatch divided by SQ_WAVES,
    last dispatch of each kernel) of the named kernels, from one or more
    rocprofv3 --pmc runs; written as a text table."""
    per = {}
    for d in dirs:
        acc = {}
        for r in _read_counter_csv(d):
            name = r.get("Kernel_Name", "")
            if not any(k in name for k in kernels):
                continue
            key = (name, r.get("Dispatch_Id", ""))
            acc.setdefault(key, {})
            c = r.get("Counter_Name", "")
            acc[key][c] = acc[key].get(c, 0.0) + float(r["Counter_Value"])
        last = {}
        for (name, did), v in acc.items():
            if name not in last or int(did or 0) > int(last[name][0] or 0):
                last[name] = (did, v)
        for name, (_, v) in last.items():
            per.setdefault(name, {}).update(v)
    lines = ["# SQ counters per wavefront (last dispatch of each kernel; counter / SQ_WAVES)",
             "# command: " + command]
    for name, v in sorted(per.items()):
        w = v.get("SQ_WAVES", 0.0) or 1.0
        lines.append(name[:110])
        lines.append("  waves %d: " % w + ", ".join("%s %.0f" % (c, x / w)
                                                  for c, x in sorted(v.items()) if c != "SQ_WAVES"))
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


PROFILE_TRACE = os.path.join(ROOT, "profiles", "kernels_bench_default.txt")


def summarize_trace(trace_dir, command, out_path=None):
    """Text summary of a rocprofv3 --kernel-trace --stats run (kernel_stats.csv):
    per kernel calls, mean and total duration, for profiles/."""
    import csv
    rows = []
    for root, _, files in os.walk(trace_dir):
        for f in files:
            if f.endswith("kernel_stats.csv"):
                with open(os.path.join(root, f)) as fh:
                    rows.extend(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 kernel trace summary (durations in microseconds)",
             "# command: " + command,
             "# step kernel source hash: " + step_kernel_hash(),
             "%-8s %12s %12s %7s  %s" % ("calls", "mean_us", "total_us", "pct", "kernel")]
    # the 40 largest, then every other step-kernel instance (the autotuner's
    # variants that lost run only its timing launches and would drop out)
    keep = rows[:40] + [r for r in rows[40:] if "k_step" in r["Name"] or "k_adj_step" in r["Name"]]
    for r in keep:
        name = r["Name"]
        if len(name) > 110:
            name = name[:110] + "..."
        lines.append("%-8s %12.2f %12.1f %7s  %s" % (r["Calls"], float(r["AverageNs"]) / 1e3,
                                                     float(r["TotalDurationNs"]) / 1e3,
                                                     r["Percentage"][:6], name))
    out_path = out_path or PROFILE_TRACE
    os.makedirs(os.path.dirname(out_path), exist_ok=True)
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def load_traffic(nodes, steps):
    """HBM bytes per step-kernel launch from committed rocprofv3 counters,
    only when they were taken on the current kernel source."""
    try:
        with open(PROFILE_PMC) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != step_kernel_hash():
        return None
    return d.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--skip-adjoint", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-annulus", action="store_true")
    ap.add_argument("--skip-lbm", action="store_true")
    ap.add_argument("--skip-tgv40", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=500)
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the 64-cloud batched leg and print its figures")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a copy of known size (for HBM counter scaling)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE)")
    ap.add_argument("--pmc-command", default="", help="command recorded in the summary")
    ap.add_argument("--summarize-traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT"),
                    help="HBM bytes per dispatch of every kernel of two --pmc runs")
    ap.add_argument("--summarize-sq", nargs="+", metavar="DIR",
                    help="per-wavefront SQ counters of --sq-kernels from --pmc runs")
    ap.add_argument("--sq-kernels", default="k_rbf,k_knn,k_adj_step")
    ap.add_argument("--sq-out", default=os.path.join(ROOT, "profiles", "sq_counters.txt"))
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR",
                    help="summarise a rocprofv3 --kernel-trace --stats run")
    ap.add_argument("--trace-out", default=None, help="where the trace summary goes")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.pmc_command, args.trace_out)
        return
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, args.pmc_command)
        return
    if args.summarize_sq:
        summarize_sq(args.summarize_sq, args.sq_kernels.split(","), args.sq_out, args.pmc_command)
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.pmc_command)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; a cloud "
              "would shard by Hilbert-ordered tile ranges with a halo exchange per step "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("RANK", "0")) != 0:
        sys.exit(0)

    if args.copy_calibration:
        copy_calibration()
    if args.batched_only:
        print(json.dumps({"batched_64_clouds": run_batched(args.batched_steps)}), flush=True)
        return
    r = run_gpu(args)
    n, K, steps = r["n"], r["K"], args.steps
    ms_step = r["ms32"] / steps
    value = n * steps / (r["ms32"] / 1e3)
    bpu = bytes_per_update(K, "f32", True)
    achieved = bpu * n / (ms_step / 1e3) / 1e9
    traffic = load_traffic(n, steps)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "timing": r["timing32"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "TGV-512: 262,144 nodes (512x512 lattice on [0,2pi)^2 jittered by "
                        "U[-0.3h,0.3h], seed 2), D2Q9 BGK tau 0.6, u0 0.01, dx = h, r^3 RBF + "
                        "degree-4 polynomials, K 30, paper stencil rule, FP32 deviation state",
            "nodes": n, "K": K, "degree": 4, "tau": 0.6, "stencil": "paper",
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_update": bpu,
            "kernel": step_kernel_name(r["tune"]["chosen"]),
            "launch_us": ms_step * 1e3,
        },
        "l2_vs_analytic": {"steps": r["l2_steps"], "fp32_u": r["l2_32"][0],
                           "fp32_vec": r["l2_32"][1]},
        "timed_state_steps": r["timed_state_steps"],
        "build_ms": r["build_ms"],
    }
    if "copy_bw" in r:
        line["copy_bandwidth"] = dict(r["copy_bw"], note="torch's device copy of 1 GiB (read "
                                      "and write): a plain streaming kernel on the same part")
    if "ms_cold" in r:
        ach_cold = bpu * n / (r["ms_cold"] / 1e3) / 1e9
        line["roofline_cache_cold"] = {
            "ms_per_step": r["ms_cold"], "achieved": ach_cold, "unit": "GB/s",
            "frac": ach_cold / HBM_PEAK_GBS,
            "note": "the same step with a second plan of the same cloud stepped in between: "
                    "twice the working set, beyond the 256 MB Infinity Cache, so every byte "
                    "comes from HBM (the headline's 310 MB per step partly stays cached)"}
    if "ms64" in r:
        line["fp64"] = {
            "value": n * steps / (r["ms64"] / 1e3), "ms_per_step": r["ms64"] / steps,
            "timing": r["timing64"],
            "roofline_frac": bytes_per_update(K, "f64", True) * n / (r["ms64"] / steps / 1e3)
            / 1e9 / HBM_PEAK_GBS,
            "l2_vs_analytic_u": r["l2_64"][0],
        }
        line["fp32_speedup_over_fp64"] = r["ms64"] / r["ms32"]
        line["fp32_vs_fp64_rel_l2"] = r["fp32_vs_fp64"]
    if "adj_ratio" in r:
        line["adjoint_over_forward"] = r["adj_ratio"]
        abpu = adjoint_bytes_per_update(K)
        ach = abpu * n / (r["adj_step_ms"] / 1e3) / 1e9
        line["adjoint_step"] = {"ms": r["adj_step_ms"], "bytes_per_update": abpu,
                                "achieved": ach, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}
        line["adjoint_rollout_500"] = r["rollout"]
        line["adjoint_rollout_500_stored"] = r["rollout_stored"]
    # local solves: n = K + M unknowns (M = 15 monomials of degree <= 4), LU-class
    # elimination 2n^3/3 plus 8 right-hand sides at 2n^2 each, per node
    nn = K + 15
    flop = n * (2.0 * nn ** 3 / 3.0 + 16.0 * nn ** 2)
    line["build"] = {"ms": r["build_ms"], "warm_builds_ms": r["build_warm_ms"],
                     "first_build_ms": r["build_cold_ms"],
                     "fp64_flop_algorithmic": flop,
                     "tflops": flop / (r["build_ms"] / 1e3) / 1e12}
    line["autotune"] = r["tune"]
    if not args.skip_lbm:
        line["lbm"] = run_lbm(args.steps, args.warmup, r["l2_steps"], r["l2_32"][0], ms_step)
    if not args.skip_tgv40:
        line["tgv40"] = run_tgv40()
    if not args.skip_annulus:
        line["annulus_490k"] = run_annulus(args.steps, args.warmup)
    if not args.skip_batched:
        line["batched_64_clouds"] = run_batched(args.batched_steps)
    if not args.no_cpu_baseline:
        log("running the FP64 oracle on the benchmarked cloud")
        errs, base = oracle_leg(r)
        line["l2_vs_oracle"] = errs
        line["l2_vs_oracle"]["note"] = (
            "velocity of the GPU state against the FP64 CPU oracle's after the same steps on "
            "the same cloud: relative L2 over all nodes and the largest per-node error over "
            "the largest oracle speed; keys are step counts (the timed state, then the full "
            "run)")
        e32 = errs.get("fp32", {}).get(str(r["l2_steps"]))
        if e32:
            line["l2_vs_oracle"]["fp32_over_method_error"] = e32["rel_l2"] / r["l2_32"][1]
        line["cpu_baseline"] = base
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
