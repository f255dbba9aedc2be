"""Throughput of the batched snake solver on one MI355X.

One step = one dt of every snake in the batch: on-device command
evaluation, chamber pressures, rest shape, prediction, the block-Jacobi
solve of every substep (to residual <= 1e-4, at most 200 iterations, by
default) and the velocity update.  The state lives in HBM between steps.

Prints one JSON line.  The headline is the uneven batch (16 384 snakes of
16 to 256 bodies, the batch the plain-versus-learned comparison is defined
on): snake-steps/s (value) and constraint-iterations/s at residual 1e-4 with
at most 200 iterations per substep, with the fraction of snakes that reach
1e-4 and the distribution of iterations per substep; no snake of this batch
reaches 1e-4 within 200 block-Jacobi iterations, and the line says so
("fixed budget, not converged").  Beside it: the dominant kernel's roofline
position (measured with HIP events on the solver's stream), the FP64 CPU
oracle timed on a bounded sample on this machine's host cores together with
the FP64 error of every GPU result on that sample, the rate at which the
uniform batch's 64-body snakes actually reach 1e-4 when the iteration cap
is lifted, the learned warm start against the zero start on its batch, the
paper's own solver (Newton with a preconditioned conjugate-residual inner
solve, FP64) and block Gauss-Seidel against block Jacobi at fixed budgets,
and the wheel carriage.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "snake-steps/s & constraint-iters/s at residual≤1e-4, plain vs NN warm-start"
# FP32 operations of the solver kernel per body-iteration, from its VALU
# counters on the uniform batch (4096 snakes of 64 bodies, every lane holds
# a body): SQ_INSTS_VALU_FLOPS_FP32 (per wave instruction: add + mul + 2 fma
# + transcendental) x 64 lanes / (262 144 bodies x 800 iterations) =
# 64 x 1.4803e9 / 2.0972e8 = 451.7 per step at the 200-iteration cap, the
# per-substep work and the final evaluation pass included (summary and
# command in profiles/k_tile_uniform4096_counters.md).
FLOP_ITER = 451.7
# hand counts of one evaluation-only pass and of the per-substep work, used
# by the Gauss-Seidel sweep count below
FLOP_EVAL = 320
FLOP_SUBSTEP = 100
PEAK_FP32 = 157.3e12       # MI355X FP32 vector (published)
# HBM bytes per launch of the solver kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs scaled by a device copy of known size (summaries in
# profiles/), keyed by workload, waves per workgroup and layout, with the digest of
# the kernel sources they were taken on; a changed kernel reports null.
MEASURED_TRAFFIC = {("uniform", 4, 1): 121.2e6, ("uneven", 4, 1): 724.9e6, ("stiff", 16, 1): 133.8e6}
TRAFFIC_SOURCES_DIGEST = "d7c930021071e3e6:06967e1b979b9c85:bb2ea3129ebb4d43:96fa7fd0a2beec66:c6116ad10c3ff82b"
PEAK_HBM = 8.0e12
# the same for the other solvers' kernels on the uniform batch (--solver),
# with the digest of their sources
# keyed by solver and workload at its default size
SOLVER_TRAFFIC = {("newton", "uniform"): (337.3e6, ("newton.hip", "lanes.h", "blocks.h", "device_math.h", "kernels.h", "fp64_recip.h"),
                                         "ffd5e28127f1372a:7d1acb2a40eb1590:06967e1b979b9c85:bb2ea3129ebb4d43:96fa7fd0a2beec66:631740f795bf42f6"),
                  ("gs", "uniform"): (52.75e6, ("gs.hip", "blocks.h", "device_math.h", "kernels.h"), "a845d97590629bbd:06967e1b979b9c85:bb2ea3129ebb4d43:96fa7fd0a2beec66"),
                  ("carriage", "uneven"): (851.5e6, ("carriage.hip", "carriage.h", "lanes.h", "blocks.h", "device_math.h", "kernels.h", "fp64_recip.h"),
                                           "e51011eec61ec901:b17d334d03f00823:7d1acb2a40eb1590:06967e1b979b9c85:bb2ea3129ebb4d43:96fa7fd0a2beec66:631740f795bf42f6"),
                  ("carriage", "uniform"): (121.5e6, ("carriage.hip", "carriage.h", "lanes.h", "blocks.h", "device_math.h", "kernels.h", "fp64_recip.h"),
                                            "e51011eec61ec901:b17d334d03f00823:7d1acb2a40eb1590:06967e1b979b9c85:bb2ea3129ebb4d43:96fa7fd0a2beec66:631740f795bf42f6")}
# Newton solver (FP64): operations per body per inner conjugate-residual
# iteration and per Newton iteration outside it (block evaluation, residual,
# rows, the two initial products, the update), counted from the compiled
# loops (add, mul = 1, fma = 2, a division or square root once); per body per
# substep outside the Newton iterations (prediction, final evaluation,
# velocities).
FLOP_PCR_ITER = 307
FLOP_NEWTON_ITER = 1050
FLOP_NEWTON_SUBSTEP = 450
# Wheel carriage (FP64): operations per segment (its joint, two wheels and
# their hinge and contact blocks) per Jacobi iteration, and per substep
# outside the iterations (pressure, rest rotation, prediction of three
# bodies, friction anchors, velocities), counted from the compiled loops as
# for the Newton solver.
FLOP_CARRIAGE_ITER = 1780
FLOP_CARRIAGE_SUBSTEP = 750
CARRIAGE_ITERS = 20
PEAK_FP64 = 78.6e12        # MI355X FP64 vector (published)
# the paper's budget (4 Newton iterations of 20 inner iterations) and two larger ones
NEWTON_BUDGETS = ((4, 20), (8, 50), (16, 50))
# block Gauss-Seidel sweeps (colour by colour over the block colouring), and
# FP32 operations per body per sweep: the residual pass and the two colour
# passes that evaluate the body's joint (FLOP_EVAL each), plus its contact
# and the five gathered updates
GS_BUDGETS = (40, 200)
FLOP_GS_SWEEP = 3 * FLOP_EVAL + 100
# learned start kept only where its residual after this many iterations is not
# larger than the zero start's (both probes' iterations count in the totals)
FALLBACK_K = 2
CONVERGING_FALLBACK_K = 400
# the same network on a batch of short snakes that fills the GPU
SATURATED_SNAKES = 65536
SATURATED_FALLBACK_K = 100
STATE_BYTES = 4 * (13 + 13 + 9 + 9)   # per body: state in/out, multipliers in/out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="uneven")
    ap.add_argument("--snakes", type=int, default=None)
    ap.add_argument("--fixed", action="store_true", help="fixed 20 iterations per substep")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--mapping", default=None,
                    help="force a mapping instead of autotuning: waves,min_seg,rows (e.g. 4,16,1)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-snakes", type=int, default=128,
                    help="snakes of the CPU-baseline sample (evenly spaced over the batch)")
    ap.add_argument("--cpu-steps", type=int, default=50, help="first steps of the CPU-baseline sample")
    ap.add_argument("--no-converged", action="store_true",
                    help="skip the leg that lifts the iteration cap until the uniform batch reaches 1e-4")
    ap.add_argument("--converged-cap", type=int, default=400000)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start comparison")
    ap.add_argument("--learned-steps", type=int, default=20)
    ap.add_argument("--no-learned-converging", action="store_true",
                    help="skip the learned-start comparison on the converging short-snake batch")
    ap.add_argument("--no-newton", action="store_true", help="skip the Newton solver comparison")
    ap.add_argument("--wheels", action="store_true",
                    help="the wheeled carriage (two wheels per segment on hinge joints), "
                         f"{CARRIAGE_ITERS} Jacobi iterations per substep")
    ap.add_argument("--no-carriage", action="store_true", help="skip the wheeled-carriage line")
    ap.add_argument("--link", action="store_true",
                    help="only the full-resolution link batch (soft links of tetrahedra and rigid frames)")
    ap.add_argument("--no-link", action="store_true", help="skip the full-resolution link line")
    ap.add_argument("--solver", default="jacobi", choices=("jacobi", "newton", "gs"),
                    help="solver of the timed loop (newton: the paper's budget, 4 x 20, FP64; "
                         "gs: block Gauss-Seidel, 40 sweeps)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three 256 MiB device copies (scale for the HBM byte counters)")
    return ap.parse_args()


def kernel_digest(files=("step.hip", "blocks.h", "device_math.h", "kernels.h", "net_inputs.h")):
    import hashlib
    csrc = os.path.join(ROOT, "paper_1904_02833_amd", "csrc")
    return ":".join(hashlib.sha256(open(os.path.join(csrc, f), "rb").read()).hexdigest()[:16] for f in files)


def learned_comparison(n_steps):
    """Learned vs zero warm start on the learned-start workload (the uneven
    batch, evaluation seed): record the solver's converged multipliers at the
    states the plain solver visits on training-seed snakes, train the
    network with the library's kernels, then time both starts."""
    import torch

    import paper_1904_02833_amd as snk
    import workloads as W
    from paper_1904_02833_amd import warmstart

    t0 = time.perf_counter()
    train_wl = W.make("uneven", n_snakes=1024, seed=2004)
    ds = warmstart.record_on_policy(train_wl, 10, stride=3, warmup_steps=6, tol=1e-6, iters=1500)
    losses = []
    net = warmstart.train(ds, epochs=4, batch=4096, lr=2e-3, log=lambda e, l: losses.append(l))
    t_train = time.perf_counter() - t0
    ev = W.make("learned")
    ev.tol, ev.iters = 1e-4, 200
    out = {"fallback_k": FALLBACK_K,
           "train": {"rows": int(ds.features.shape[0]), "seconds": t_train, "loss_by_epoch": losses,
                     "teacher": "tolerance 1e-6 (at most 1500 iterations), first substep of states "
                                "visited by the plain solver",
                     "step": training_step_rate(net, ds)}}
    for name in ("plain", "learned"):
        sim = (snk.Sim(ev, autotune=1) if name == "plain"
               else warmstart.learned_sim(ev, net, autotune=1, mlp_fallback_k=FALLBACK_K))
        sim.step(5)
        torch.cuda.synchronize()
        r0 = sim.read("iters_total")["iters_total"].copy()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        for _ in range(n_steps):
            sim.step(1)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        r = sim.read("iters_total", "residual", "status")
        its = (r["iters_total"] - r0).astype(np.float64)
        B = ev.bodies.astype(np.float64)
        out[name] = {"snake_steps_per_s": ev.n_snakes * n_steps / (ms / 1e3),
                     "constraint_iters_per_s": float(np.sum((9 * B - 6) * its)) / (ms / 1e3),
                     "ms_per_step": ms / n_steps,
                     "mean_iters_per_substep": float(its.sum() / (ev.n_snakes * n_steps * ev.substeps)),
                     **iteration_stats(its, ev.substeps, n_steps, r["status"], r["residual"], ev.tol, ev.iters),
                     "fell_back_last_step": int(np.sum((r["status"] & 4) != 0))}
        sim.close()
    out["workload"] = (f"learned: the uneven batch's shape and draws, evaluation seed, {ev.n_snakes} snakes, "
                       f"residual<=1e-4 or at most {ev.iters} iterations per substep")
    out["gain"] = learned_gain(out["plain"], out["learned"])
    return out


# network arithmetic per sample: forward 2 (32*64 + 64*64 + 64*3) flop;
# backward the weight gradients of all three layers and the input gradients
# of layers 3 and 2, 2 (32*64 + 2*64*64 + 2*64*3) flop
NET_FWD_FLOP = 2 * (32 * 64 + 64 * 64 + 64 * 3)
NET_BWD_FLOP = 2 * (32 * 64 + 2 * 64 * 64 + 2 * 64 * 3)
PEAK_BF16 = 2.5e15        # MI355X dense BF16 MFMA (published)


def training_step_rate(net, ds, batch=4096, n=50):
    """One training step of the network (gradient of a 4096-sample batch,
    the ordered reduction of its chunk rows, Adam) timed with HIP events on
    the stream the library launches on, against the BF16 MFMA peak."""
    import torch

    x, t = ds.features[:batch], ds.targets[:batch]
    lr = 0.0   # parameters unchanged: the timed steps leave the trained network as it is
    for _ in range(5):
        g, _ = net.grad(x, t)
        net.adam(g, lr=lr)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(n):
        g, _ = net.grad(x, t)
        net.adam(g, lr=lr)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / n
    flop = x.shape[0] * (NET_FWD_FLOP + NET_BWD_FLOP)
    return {"batch": int(x.shape[0]), "us_per_step": us, "samples_per_s": x.shape[0] / (us * 1e-6),
            "roofline": {"bound": "mfma", "achieved": flop / (us * 1e-6) / 1e12, "peak": PEAK_BF16 / 1e12,
                         "unit": "TFLOP/s", "frac": flop / (us * 1e-6) / PEAK_BF16,
                         "flop_per_sample": NET_FWD_FLOP + NET_BWD_FLOP}}


def learned_gain(plain, learned, margin=0.02):
    """Whether the learned start takes fewer iterations and gives more
    snake-steps/s than the plain one; a rate counts as higher only beyond
    the run-to-run spread of a step time on one GPU (about 2 %)."""
    ratio = learned["snake_steps_per_s"] / plain["snake_steps_per_s"]
    return {"fewer_iterations": learned["mean_iters_per_substep"] < plain["mean_iters_per_substep"],
            "snake_steps_per_s_ratio": ratio,
            "more_snake_steps_per_s": ratio > 1.0 + margin}


def learned_converging(n_steps=6):
    """Learned vs zero start where the solve converges within its budget:
    the short-snake batch (6 or 8 bodies), residual 1e-4 with at most 30 000
    iterations, at its default size (4096 snakes: the step time follows the
    slowest snake) and on a batch that fills the GPU (65 536 snakes).  The
    network learns the converged multipliers (tolerance 1e-7) at the states
    of a converged trajectory of training-seed snakes; both starts then run
    from the same converged state of the evaluation snakes, the learned one
    kept only where its residual after k iterations (CONVERGING_FALLBACK_K,
    SATURATED_FALLBACK_K) is not larger than the zero start's."""
    import torch

    import paper_1904_02833_amd as snk
    import workloads as W
    from paper_1904_02833_amd import warmstart

    t0 = time.perf_counter()
    ds = warmstart.record(W.make("short", seed=2005), 8, tol=1e-7, iters=60000)
    losses = []
    net = warmstart.train(ds, epochs=12, batch=4096, lr=2e-3, log=lambda e, l: losses.append(l))
    t_train = time.perf_counter() - t0
    ev = W.make("short")
    ev.tol, ev.iters = 1e-4, 30000
    lead = snk.Sim(ev, tol=1e-7, iters=60000)
    lead.step(6)
    state = lead.read()
    lead.close()
    out = {"workload": f"short: {ev.n_snakes} snakes of 6 or 8 bodies, residual<=1e-4, max {ev.iters} iterations",
           "fallback_k": CONVERGING_FALLBACK_K,
           "train": {"rows": int(ds.features.shape[0]), "seconds": t_train, "loss_by_epoch": losses}}

    def compare(ev, state, k, n_steps, **mapping):
        res = {}
        for name in ("plain", "learned"):
            sim = (snk.Sim(ev, **mapping) if name == "plain"
                   else warmstart.learned_sim(ev, net, mlp_fallback_k=k, **mapping))
            sim.write(**state)
            sim.step(1)
            torch.cuda.synchronize()
            r0 = sim.read("iters_total")["iters_total"].copy()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(sim.stream)
            for _ in range(n_steps):
                sim.step(1)
            e1.record(sim.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / n_steps
            r = sim.read("iters_total", "residual", "status")
            its = (r["iters_total"] - r0) / (n_steps * ev.substeps)
            res[name] = {"snake_steps_per_s": ev.n_snakes / (ms / 1e3), "ms_per_step": ms,
                         "mean_iters_per_substep": float(its.mean()),
                         "median_iters_per_substep": float(np.median(its)),
                         "not_converged_last_step": int(np.sum((r["status"] & 2) != 0)),
                         "fell_back_last_step": int(np.sum((r["status"] & 4) != 0))}
            sim.close()
        res["gain"] = learned_gain(res["plain"], res["learned"])
        return res

    out.update(compare(ev, state, CONVERGING_FALLBACK_K, n_steps))
    # A batch that fills the GPU (half rows: two snakes per 16-lane row, 8
    # waves per SIMD slot): the step time then follows the mean iteration
    # count rather than the slowest snake's.  Both forms take the same mapping.
    big = W.make("short", n_snakes=SATURATED_SNAKES)
    big.tol, big.iters = 1e-4, 30000
    half_rows = dict(map_waves=4, map_rows=2)
    lead = snk.Sim(big, tol=1e-7, iters=60000, **half_rows)
    lead.step(6)
    big_state = lead.read()
    lead.close()
    out["saturated"] = {"workload": f"short: {big.n_snakes} snakes, residual<=1e-4, max {big.iters} iterations, "
                                    "half rows",
                        "fallback_k": SATURATED_FALLBACK_K,
                        **compare(big, big_state, SATURATED_FALLBACK_K, 4, **half_rows)}
    return out


def newton_comparison(wl, n_steps=5):
    """The paper's own solver (Newton iterations, each solving the
    Schur-complement system with preconditioned conjugate-residual
    iterations, FP64) and block Gauss-Seidel over the block colouring (FP32)
    against block Jacobi (FP32) on the same batch, from the same state (20
    plain steps in), at several fixed budgets: time per step and the
    residual each reaches."""
    import torch

    import paper_1904_02833_amd as snk

    lead = snk.Sim(wl)
    lead.step(20)
    state = lead.read()
    lead.close()
    B = wl.bodies.astype(np.float64)
    rows = []

    def run(label, **kw):
        sim = snk.Sim(wl, **kw)
        sim.write(**state)
        sim.step(1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        for _ in range(n_steps):
            sim.step(1)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n_steps
        r = sim.read("residual", "status")
        sim.close()
        row = {"solver": label, "ms_per_step": ms, "snake_steps_per_s": wl.n_snakes / (ms / 1e3),
               "residual_last_step": {"median": float(np.median(r["residual"])),
                                      "p99": float(np.percentile(r["residual"], 99)),
                                      "max": float(np.max(r["residual"]))},
               "nonfinite_snakes": int(np.sum((r["status"] & 1) != 0))}
        if kw.get("solver") == snk.SOLVER_NEWTON:
            ni, npc = kw["newton_iters"], kw["pcr_iters"]
            per_body = wl.substeps * (ni * (FLOP_NEWTON_ITER + npc * FLOP_PCR_ITER) + FLOP_NEWTON_SUBSTEP)
            ach = float(B.sum()) * per_body / (ms / 1e3)
            row["roofline"] = {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_FP64 / 1e12,
                               "unit": "TFLOP/s", "frac": ach / PEAK_FP64, "traffic": None,
                               "kernel": "k_newton<SEG>", "dtype": "f64"}
        rows.append(row)

    # Jacobi in the launch shape the autotuner picks, as on the headline line
    run("jacobi, 200 iterations", tol=0.0, iters=200, autotune=1)
    run("jacobi, 2000 iterations", tol=0.0, iters=2000, autotune=1)
    for sweeps in GS_BUDGETS:
        run(f"gauss-seidel, {sweeps} sweeps", solver=snk.SOLVER_GS, tol=0.0, iters=sweeps)
    for ni, npc in NEWTON_BUDGETS:
        run(f"newton, {ni} x {npc} inner iterations", solver=snk.SOLVER_NEWTON, newton_iters=ni, pcr_iters=npc,
            tol=0.0)
    ni, npc = NEWTON_BUDGETS[0]
    run(f"newton, {ni} x {npc} inner iterations, previous multipliers", solver=snk.SOLVER_NEWTON,
        newton_iters=ni, pcr_iters=npc, tol=0.0, warm_start=snk.WARM_PREV)
    for ni, npc in NEWTON_BUDGETS[:2]:
        run(f"newton, {ni} x {npc} inner iterations, best iterate kept", solver=snk.SOLVER_NEWTON,
            newton_iters=ni, pcr_iters=npc, tol=0.0, newton_keep_best=1)
    return {"workload": f"{wl.name}: {wl.n_snakes} snakes, {int(B.sum())} bodies, {wl.substeps} substeps, "
                        "fixed budgets from the state after 20 plain steps",
            "rows": rows}


def carriage_run(wl, n_steps=5, iters=CARRIAGE_ITERS, default_size=True):
    """The batch on wheels (two per segment on hinge joints, FP64 Jacobi
    iterations) from the state after 20 steps on wheels: time per step, the
    residual reached and the kernel's FP64 throughput."""
    import torch

    import paper_1904_02833_amd as snk

    cw = wl.take(np.arange(wl.n_snakes))
    cw.flags = cw.flags | snk.FLAG_WHEELS
    cw.tol, cw.iters = 0.0, iters
    sim = snk.Sim(cw)
    sim.step(20)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    for _ in range(n_steps):
        sim.step(1)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / n_steps
    r = sim.read("residual", "status")
    sim.close()
    B = float(cw.bodies.sum())
    ach = B * cw.substeps * (iters * FLOP_CARRIAGE_ITER + FLOP_CARRIAGE_SUBSTEP) / (ms / 1e3)
    traffic = None
    key = ("carriage", wl.name)
    if key in SOLVER_TRAFFIC and default_size:
        t, files, digest = SOLVER_TRAFFIC[key]
        traffic = t if kernel_digest(files) == digest else None
    return {"workload": f"{wl.name} on wheels: {cw.n_snakes} snakes, {int(B)} segments, {int(2 * B)} wheels, "
                        f"{cw.substeps} substeps, {iters} iterations",
            "ms_per_step": ms, "snake_steps_per_s": cw.n_snakes / (ms / 1e3),
            "residual_last_step": {"median": float(np.median(r["residual"])),
                                   "max": float(np.max(r["residual"]))},
            "nonfinite_snakes": int(np.sum((r["status"] & 1) != 0)),
            "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                         "frac": ach / PEAK_FP64, "traffic": traffic, "kernel": "k_carriage<64>", "dtype": "f64",
                         "flop_per_segment_iter": FLOP_CARRIAGE_ITER}}


# Full-resolution link (FP32): operations of the link kernel per
# link-iteration (288 elements, 196 distance rows, 18 attachments and the
# gather and contact of 117 particles, the elements dominating), from its
# VALU counters on the link batch (k_link dispatches only):
# SQ_INSTS_VALU_FLOPS_FP32 x 64 lanes / (2048 snakes x 4 links x 80
# iterations) = 64 x 1.86413e9 / 655 360 (profiles/k_link_link2048x4.md).
# HBM bytes per launch from FETCH_SIZE and WRITE_SIZE on that batch, with
# the digest of the kernel's sources.
LINK_SNAKES = 2048
LINK_STEPS = 10
LINK_FLOP_ITER = 182_040
LINK_TRAFFIC = (436.2e6, 2048, ("link.hip", "device_math.h"), "1b641d59d387afe6:bb2ea3129ebb4d43")


def link_run(n_snakes=LINK_SNAKES, n_steps=LINK_STEPS, iters=20):
    """The link batch: snakes of four soft links on the procedural
    13-section tetrahedral mesh (117 particles, 288 elements per link) and
    five rigid frames, 4 substeps x `iters` block-Jacobi iterations, drawn
    piecewise-constant chamber commands set from a device array every step.
    Time per step, the residual reached, and the element-iterations per
    second."""
    import torch

    import workloads as W
    from paper_1904_02833_amd.link import LinkSim

    wl = W.make_link(n_snakes, n_links=4)
    wl.iters = iters
    cmds = torch.as_tensor(W.link_commands(wl, 20 + n_steps), dtype=torch.float32, device="cuda")
    sim = LinkSim(wl)
    for n in range(20):
        sim.set_commands(cmds[n])
        sim.step(1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    for n in range(20, 20 + n_steps):
        sim.set_commands(cmds[n])
        sim.step(1)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / n_steps
    r = sim.read("residual", "status", "iters")
    sim.close()
    tets = n_snakes * wl.n_links * wl.n_tets
    its = float(np.mean(r["iters"]))
    # algorithmic HBM bytes per snake-step: particle positions and velocities
    # in; positions, velocities, contact multipliers out; frame states in and
    # out; pressures and commands; every multiplier out; the four status words
    L, P1 = wl.n_links, wl.per_link
    D1 = (wl.sections - 1) * (wl.ring + 1) + (wl.sections - 2) * wl.ring
    A1 = 2 * (wl.ring + 1)
    per_snake = (L * P1 * (24 + 36) + (L + 1) * 2 * 52 + L * (8 + 4 + 8)
                 + L * (24 * wl.n_tets + 4 * D1 + 12 * A1) + 16)
    flops = LINK_FLOP_ITER * n_snakes * L * its / (ms / 1e3)
    t, n_ref, files, digest = LINK_TRAFFIC
    traffic = t if (n_snakes == n_ref and kernel_digest(files) == digest) else None
    return {"workload": f"link: {n_snakes} snakes x {wl.n_links} soft links ({wl.per_link} particles, {wl.n_tets} "
                        f"tetrahedra per link) and {wl.n_links + 1} rigid frames, {wl.substeps} substeps x {iters} "
                        "iterations, drawn chamber commands",
            "ms_per_step": ms, "snake_steps_per_s": n_snakes / (ms / 1e3),
            "element_iters_per_s": tets * its / (ms / 1e3),
            "iters_per_step": its,
            "residual_last_step": {"median": float(np.median(r["residual"])),
                                   "max": float(np.max(r["residual"]))},
            "nonfinite_snakes": int(np.sum((r["status"] & 1) != 0)),
            "roofline": {"bound": "alu", "achieved": flops / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                         "frac": flops / PEAK_FP32, "traffic": traffic, "kernel": "k_link", "dtype": "f32",
                         "flop_per_link_iter": LINK_FLOP_ITER,
                         "hbm_bytes_algorithmic": per_snake * n_snakes,
                         "hbm_frac_algorithmic": per_snake * n_snakes / (ms / 1e3) / PEAK_HBM}}


def host_cores():
    """Threads the oracle runs on: the CPUs this process may use, at most 16
    (the host share of one GPU on the benchmark machines, whatever the
    machine's own core count; both numbers are reported)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail)), avail


# first-steps samples of the other batches for the CPU baseline: snakes, steps
# (the stiff batch at 10 steps keeps the baseline within a minute)
CPU_OTHER = {"uniform": (64, 50), "stiff": (4, 10)}   # stiff: 1.2 s per snake-step


def cpu_baseline(wl, n_snakes, n_steps, gpu_kw):
    """The FP64 oracle as it stands, timed on this machine's host cores:
    (1) the single-snake workload in full (600 steps, 4 substeps x 20
    iterations), one thread; (2) the first n_steps steps of n_snakes snakes
    spread evenly over the timed batch, its settings, snakes split over the
    host cores; (3) the same for the uniform and stiff batches (CPU_OTHER).
    The value is (2)'s snake-steps/s.  Then both sides take one more
    substep of the (2) sample from the oracle's state rounded to FP32, and
    the GPU's results are compared with the oracle's (the FP64 error of
    every result: positions, velocities, angular velocities, multipliers)."""
    import oracle
    import workloads as W
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import advance_both, compare, rounded_state

    threads, avail = host_cores()
    single = W.make("single")
    o1 = oracle.Oracle(single)
    t0 = time.perf_counter()
    o1.run(single.n_steps, threads=1)
    t_single = time.perf_counter() - t0

    pick = np.unique(np.linspace(0, wl.n_snakes - 1, min(n_snakes, wl.n_snakes)).round().astype(np.int64))
    sub = wl.take(pick)
    o = oracle.Oracle(sub)
    t0 = time.perf_counter()
    o.run(n_steps, threads=threads)
    dt = time.perf_counter() - t0
    out = {"value": sub.n_snakes * n_steps / dt, "unit": "snake-steps/s", "cores": threads,
           "host_cpus_available": avail, "kind": "oracle",
           "sample": f"first {n_steps} steps of {sub.n_snakes} of the {wl.n_snakes} snakes (evenly spaced "
                     f"by index, {int(sub.bodies.sum())} bodies), the timed batch's settings, FP64 C oracle "
                     f"on {threads} threads, {dt:.1f} s wall",
           "constraint_iters_per_s": float(np.sum((9 * sub.bodies - 6) * o.iters_total) / dt),
           "single_snake_full": {"workload": f"single: 1 snake of 64 bodies, {single.n_steps} steps, "
                                             f"{single.substeps} substeps x {single.iters} iterations",
                                 "snake_steps_per_s": single.n_steps / t_single, "seconds": t_single,
                                 "cores": 1}}
    others = {}
    for name, (ns, nst) in CPU_OTHER.items():
        ow = W.make(name)
        if name == "uniform":
            ow.tol, ow.iters = wl.tol, wl.iters
        ow = ow.take(np.unique(np.linspace(0, ow.n_snakes - 1, ns).round().astype(np.int64)))
        oo = oracle.Oracle(ow)
        t0 = time.perf_counter()
        oo.run(nst, threads=threads)
        t = time.perf_counter() - t0
        others[name] = {"snake_steps_per_s": ow.n_snakes * nst / t, "seconds": t,
                        "sample": f"first {nst} steps of {ow.n_snakes} snakes ({int(ow.bodies.sum())} bodies), "
                                  f"residual<=1e-4 or at most {ow.iters} iterations" if ow.tol > 0 else
                                  f"first {nst} steps of {ow.n_snakes} snakes, {ow.iters} iterations"}
    out["other_batches"] = others
    # the FP64 network's inference cost for the learned start (one thread):
    # rows of 32 inputs through 32 -> 64 -> 64 -> 3 with exact-erf GELU
    rng = np.random.default_rng(7)
    n_rows = 1 << 16
    params = rng.normal(scale=0.2, size=oracle.mlp_param_count())
    xs = rng.normal(size=(n_rows, 32))
    t0 = time.perf_counter()
    oracle.mlp_forward(params, np.zeros(32), np.ones(32), xs)
    t_net = time.perf_counter() - t0
    rows_uneven = 2 * int(np.sum(wl.bodies - 1))
    out["network_inference"] = {"rows_per_s": n_rows / t_net, "seconds": t_net, "cores": 1,
                                "sample": f"{n_rows} rows of 32 inputs, random weights of the network's shape, "
                                          "FP64 C oracle with exact-erf GELU",
                                "per_substep_s_timed_batch": rows_uneven / (n_rows / t_net),
                                "rows_per_substep_timed_batch": rows_uneven}
    o.commands()
    oo, g = advance_both(sub, rounded_state(o), threads=threads, **gpu_kw)
    err = compare(oo, g, np.asarray(sub.mu, np.float64))
    out["fp64_error"] = {
        "protocol": "one substep of the sample from the oracle's state rounded to FP32, GPU (FP32) "
                    "against the FP64 oracle; positions relative to the snake's extent, velocities "
                    "to max(|v|, g h) and max(|w|, g h / L), multipliers per block type to their "
                    "largest magnitude (floor m g h^2, bend m g h^2 L)",
        **{k: {"max": float(np.max(v)), "p99": float(np.percentile(v, 99))}
           for k, v in err.items() if k != "branch"},
        "contact_branch_mismatches": int(err["branch"].sum()),
        "bodies": int(sub.bodies.sum())}
    return out


def iteration_stats(its, substeps, n_steps, status, residual, tol, cap):
    """Per-snake iterations per substep over the timed steps, the fraction
    of snakes whose last step reached the tolerance in every substep, and
    the last step's residuals."""
    per = its / (substeps * n_steps)
    conv = (status & 2) == 0
    st = {"tol": tol, "max_iters": cap,
          "converged_frac_last_step": float(conv.mean()),
          "iters_per_substep": {"mean": float(per.mean()), "median": float(np.median(per)),
                                "p99": float(np.percentile(per, 99)), "max": float(per.max())},
          "residual_last_step": {"median": float(np.median(residual)),
                                 "p99": float(np.percentile(residual, 99)), "max": float(np.max(residual))}}
    st["label"] = ("converged" if conv.all() else
                   "fixed budget, not converged" if not conv.any() else "partly converged")
    return st


def converged_run(name="uniform", n_steps=2, cap=400000):
    """The batch from rest with the iteration cap lifted until its snakes
    reach residual 1e-4 (or stall at FP32's floor): snake-steps/s and
    constraint-iterations/s at the tolerance, with the iterations it took."""
    import torch

    import paper_1904_02833_amd as snk
    import workloads as W

    wl = W.make(name)
    wl.tol, wl.iters = 1e-4, cap
    sim = snk.Sim(wl, use_graph=1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res, ms_steps, its_all = [], [], []
    for n in range(n_steps):
        before = sim.read("iters_total")["iters_total"].copy()
        e0.record(sim.stream)
        sim.step(1)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        ms_steps.append(e0.elapsed_time(e1))
        r = sim.read("iters_total", "residual", "status")
        its_all.append((r["iters_total"] - before).astype(np.float64))
        res.append(r)
        print(f"[converged {name}] step {n}: {ms_steps[-1]:.0f} ms, "
              f"converged {float(np.mean((r['status'] & 2) == 0)):.3f}", file=sys.stderr, flush=True)
    sim.close()
    its = np.sum(its_all, axis=0)
    ms = float(np.sum(ms_steps))
    B = wl.bodies.astype(np.float64)
    last = res[-1]
    return {"workload": f"{name}: {wl.n_snakes} snakes, {int(B.sum())} bodies, {wl.substeps} substeps, "
                        f"from rest, residual<=1e-4 with at most {cap} iterations per substep",
            "steps": n_steps, "ms_per_step": ms / n_steps, "ms_each_step": ms_steps,
            "snake_steps_per_s": wl.n_snakes * n_steps / (ms / 1e3),
            "constraint_iters_per_s": float(np.sum((9 * B - 6) * its)) / (ms / 1e3),
            **iteration_stats(its, wl.substeps, n_steps, last["status"], last["residual"], 1e-4, cap)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1 "
                          "(snakes are independent: several GPUs would each take a share of the snakes, "
                          "one process per GPU, with no exchange during a step)"}))
        sys.exit(2)
    import torch

    if args.copy_calibration:
        n = 256 << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": n, "dispatches": 3}), flush=True)
        return

    import paper_1904_02833_amd as snk
    import workloads as W

    if args.link:
        row = link_run(n_snakes=args.snakes or LINK_SNAKES, n_steps=args.steps)
        out = {"metric": "link snake-steps/s", "value": row["snake_steps_per_s"], "unit": "snake-steps/s",
               "n_gpus": 1, "steps": args.steps, "warmup": 20, "ms_per_step": row["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": row["workload"]}, **{k: v for k, v in row.items() if k != "workload"}}
        print(json.dumps(out), flush=True)
        return
    wl = W.make(args.workload, n_snakes=args.snakes)
    if args.wheels:
        if args.solver != "jacobi":
            raise SystemExit("--wheels takes the Jacobi solver")
        row = carriage_run(wl, n_steps=args.steps)
        out = {"metric": "wheel-carriage snake-steps/s", "value": row["snake_steps_per_s"],
               "unit": "snake-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": 20,
               "ms_per_step": row["ms_per_step"], "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": row["workload"]}, "roofline": row["roofline"],
               "residual_last_step": row["residual_last_step"]}
        print(json.dumps(out), flush=True)
        return
    if args.fixed:
        wl.tol, wl.iters = 0.0, 20
    else:
        wl.tol, wl.iters = 1e-4, 200
    newton = args.solver == "newton"
    gs = args.solver == "gs"
    gpu_kw = {}
    if gs:
        wl.tol, wl.iters = 0.0, GS_BUDGETS[0]
        gpu_kw = dict(solver=snk.SOLVER_GS)
        sim = snk.Sim(wl, use_graph=1, **gpu_kw)
    elif newton:
        wl.tol = 0.0
        ni, npc = NEWTON_BUDGETS[0]
        gpu_kw = dict(solver=snk.SOLVER_NEWTON, newton_iters=ni, pcr_iters=npc)
        sim = snk.Sim(wl, use_graph=1, **gpu_kw)
    elif args.mapping:
        mw, ms, mr = (int(v) for v in args.mapping.split(","))
        sim = snk.Sim(wl, use_graph=1, autotune=0, map_waves=mw, map_min_seg=ms, map_rows=mr)
    else:
        sim = snk.Sim(wl, use_graph=1, autotune=0 if args.no_autotune else 1)
    stream = sim.stream
    for _ in range(args.warmup):
        sim.step(1)
    torch.cuda.synchronize()
    before = sim.read("iters_total")["iters_total"].copy()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        sim.step(1)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    r = sim.read("iters_total", "residual", "status")
    its = (r["iters_total"] - before).astype(np.float64)
    B = wl.bodies.astype(np.float64)
    rows = 9 * B - 6
    secs = ms / 1e3
    snake_steps = wl.n_snakes * args.steps / secs
    citers = float(np.sum(rows * its)) / secs
    flops = float(np.sum(B * its)) * FLOP_ITER
    if newton:
        flops = float(B.sum()) * args.steps * wl.substeps * (
            ni * (FLOP_NEWTON_ITER + npc * FLOP_PCR_ITER) + FLOP_NEWTON_SUBSTEP)
    elif gs:
        flops = float(np.sum(B * (its * FLOP_GS_SWEEP + args.steps * wl.substeps * (FLOP_EVAL + FLOP_SUBSTEP))))
    per_launch_ms = ms / args.steps
    achieved = flops / args.steps / (per_launch_ms / 1e3)
    hbm_bytes = float(B.sum()) * STATE_BYTES
    traffic = (MEASURED_TRAFFIC.get((args.workload, sim.mapping["waves"], sim.mapping["rows"]))
               if args.snakes is None else None)
    if newton or gs:
        traffic = None
        if (args.solver, args.workload) in SOLVER_TRAFFIC and args.snakes is None:
            t, files, digest = SOLVER_TRAFFIC[(args.solver, args.workload)]
            traffic = t if kernel_digest(files) == digest else None
    elif traffic is not None and kernel_digest() != TRAFFIC_SOURCES_DIGEST:
        traffic = None
    conv = iteration_stats(its, wl.substeps, args.steps, r["status"], r["residual"], wl.tol, wl.iters)
    budget = (f"Newton {ni} x {npc} inner iterations" if newton
              else f"Gauss-Seidel {wl.iters} sweeps" if gs
              else "20 iterations" if args.fixed
              else f"residual<=1e-4 or at most 200 iterations per substep ({conv['label']}: "
                   f"{conv['converged_frac_last_step']:.3f} of the snakes reach 1e-4)")
    out = {
        "metric": METRIC,
        "value": snake_steps,
        "unit": "snake-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per_launch_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if newton else "f32",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.n_snakes} snakes of {int(B.min())}..{int(B.max())} bodies, "
                               f"{int(B.sum())} bodies, {wl.substeps} substeps, {budget}, plain (zero warm start)",
                   "snakes": wl.n_snakes, "bodies": int(B.sum()), "substeps": wl.substeps,
                   "tol": wl.tol, "max_iters": wl.iters},
        "constraint_iters_per_s": citers,
        "convergence": conv,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": (PEAK_FP64 if newton else PEAK_FP32) / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / (PEAK_FP64 if newton else PEAK_FP32), "traffic": traffic,
                     "kernel": "k_newton<64>" if newton else "k_gs<64>" if gs
                     else f"k_tile<{sim.mapping['waves']}, 0, {sim.mapping['rows']}>",
                     "mapping": sim.mapping,
                     "flop_per_body_iter": FLOP_PCR_ITER if newton else FLOP_GS_SWEEP if gs else FLOP_ITER,
                     "hbm_bytes_algorithmic": hbm_bytes,
                     "hbm_frac_algorithmic": hbm_bytes / (per_launch_ms / 1e3) / PEAK_HBM},
    }
    sim.close()
    print(f"[bench] headline {snake_steps:.4g} snake-steps/s, {per_launch_ms:.3f} ms per step",
          file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_snakes, args.cpu_steps, gpu_kw)
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)
    if not args.no_converged:
        out["converged_at_tolerance"] = converged_run("uniform", cap=args.converged_cap)
    if not args.no_learned:
        out["learned_warm_start"] = learned_comparison(args.learned_steps)
        print("[bench] learned comparison done", file=sys.stderr, flush=True)
        if not args.no_learned_converging:
            out["learned_warm_start_converging"] = learned_converging()
            print("[bench] learned converging done", file=sys.stderr, flush=True)
    if not args.no_newton:
        out["newton_pcr"] = newton_comparison(wl)
        print("[bench] solver comparison done", file=sys.stderr, flush=True)
    if not args.no_carriage:
        out["wheel_carriage"] = carriage_run(wl, default_size=args.snakes is None)
    if not args.no_link:
        out["full_resolution_link"] = link_run()
        print("[bench] link done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
