"""GPU block Gauss-Seidel (FP32, colour by colour over the index work's
greedy block colouring) against the FP64 oracle's Gauss-Seidel solver, per
the substep protocol of tests/parity.py: positions to 1e-5, velocities and
multipliers to 1e-4 relative per block type (the friction multipliers to
twice the oracle's own spread under a one-ulp input nudge, 1e-4 to 0.28 by
case: the sequential sweep's friction is that sensitive), contacts whose active set or stick/slip branch differs
between the precisions counted apart (at most 2 % of bodies).  Whole steps
are checked substep by substep.  Lane classes 8 to 1024."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import LAM_TOL, POS_TOL, VEL_TOL, advance_both, compare, load_oracle, rounded_state

pytestmark = pytest.mark.gpu
snk = pytest.importorskip("paper_1904_02833_amd")

GS = dict(solver=snk.SOLVER_GS)


def state_after(wl, steps, **over):
    o = oracle.Oracle(wl, **over)
    o.run(steps, threads=8)
    o.commands()
    return rounded_state(o)


def gs_parity(tag, wl, st, cond_gate=("lam_t",), **over):
    """Advance the rounded state st one substep on both sides: positions to
    1e-5, velocities and multipliers to 1e-4 per type, sweep counts equal.
    The spread of the FP64 oracle's own result when its input positions
    move by one FP32 ulp (the conditioning of the substep) is printed beside
    the errors; the block types named in cond_gate (the friction
    multipliers) are gated at twice that spread where it exceeds 1e-4.  A
    Gauss-Seidel sweep carries every contact's friction update into the
    next block's state at once, and the sticking contacts' friction of one
    substep moves by 1e-4 to 6.6e-3 of its scale under a one-ulp input
    nudge (0.28 on the near-rigid stiff chains, where compliances of 1e-8
    decide the split of the friction among sticking contacts); the GPU's
    errors sit at 4e-5 to 4e-4, inside that."""
    o, g = advance_both(wl, st, **GS, **over)
    kw = dict(controller=W.CTRL_EXTERNAL, solver=oracle.SOLVER_GS, dt=wl.dt / wl.substeps, substeps=1, **over)
    o2 = oracle.Oracle(wl, **kw)
    nudged = dict(st)
    nudged["x"] = np.nextafter(st["x"].astype(np.float32), np.float32(np.inf)).astype(np.float64)
    load_oracle(o2, nudged)
    o2.run(1, threads=8)
    mu = np.asarray(wl.mu, np.float64)
    spread = compare(o, dict(x=o2.x, lam_j=o2.lam_j, lam_c=o2.lam_c), mu)
    err = compare(o, g, mu)
    keys = ("lam_s", "lam_b", "lam_n", "lam_t")
    print(f"\n[{tag}] worst", {k: float(err[k].max()) for k in err if k != "branch"},
          "FP64 1-ulp spread", {k: float(spread[k].max()) for k in keys},
          "branch mismatches", int(err["branch"].sum()), flush=True)
    assert np.array_equal(np.asarray(g["iters"]), o.iters)
    assert err["pos"].max() <= POS_TOL
    for k in ("vel", "angvel"):
        assert err[k].max() <= VEL_TOL, k
    for k in keys:
        gate = max(LAM_TOL, 2 * spread[k].max()) if k in cond_gate else LAM_TOL
        assert err[k].max() <= gate, (k, float(err[k].max()), gate)
    assert err["branch"].sum() <= 0.02 * int(wl.bodies.sum())
    return o, g


def short_uneven(n, max_B=64):
    wl = W.make("uneven", n_snakes=4 * n)
    return wl.take(np.nonzero(wl.bodies <= max_B)[0][:n])


@pytest.mark.parametrize("name", ["uniform", "uneven_short", "uneven", "short"])
def test_gs_substep_parity(name):
    wl = {"uniform": lambda: W.make("uniform", n_snakes=48), "uneven_short": lambda: short_uneven(120),
          "uneven": lambda: W.make("uneven", n_snakes=40), "short": lambda: W.make("short", n_snakes=64)}[name]()
    gs_parity(f"gs substep {name}", wl, state_after(wl, 20))


def test_gs_step_parity_uneven():
    """A whole step (four substeps), substep by substep: the one-launch
    step equals four one-substep launches bit for bit, and each of those is
    held to the per-substep gates against the oracle from the GPU's own
    state before it (friction multipliers at twice the oracle's one-ulp
    spread, as in every Gauss-Seidel case)."""
    from parity import chained_substeps

    wl = W.make("uneven", n_snakes=24)
    orc = dict(solver=oracle.SOLVER_GS)
    steps = chained_substeps(wl, state_after(wl, 10), gpu_over=GS, orc_over=orc)
    mu = np.asarray(wl.mu, np.float64)
    for k, (o, g, st) in enumerate(steps):
        o2 = oracle.Oracle(wl, controller=W.CTRL_EXTERNAL, dt=wl.dt / wl.substeps, substeps=1, **orc)
        load_oracle(o2, dict(st, x=np.nextafter(st["x"].astype(np.float32), np.float32(np.inf)).astype(np.float64)))
        o2.run(1, threads=8)
        spread = compare(o, dict(x=o2.x, lam_j=o2.lam_j, lam_c=o2.lam_c), mu)
        err = compare(o, g, mu)
        print(f"\n[gs step uneven, substep {k}] worst", {q: float(err[q].max()) for q in err if q != "branch"},
              "FP64 1-ulp spread", {q: float(spread[q].max()) for q in ("lam_s", "lam_b", "lam_n", "lam_t")},
              "branch mismatches", int(err["branch"].sum()), flush=True)
        assert np.array_equal(np.asarray(g["iters"]), o.iters)
        assert err["pos"].max() <= POS_TOL
        for q in ("vel", "angvel", "lam_s", "lam_b", "lam_n"):
            assert err[q].max() <= LAM_TOL, (k, q, float(err[q].max()))
        assert err["lam_t"].max() <= max(LAM_TOL, 2 * spread["lam_t"].max()), (k, float(err["lam_t"].max()))
        assert err["branch"].sum() <= 0.02 * int(wl.bodies.sum())


def test_gs_stiff_1024_lanes():
    wl = W.make("stiff", n_snakes=2)
    gs_parity("gs stiff", wl, state_after(wl, 4))


def test_gs_tiny_odd_sizes_and_fixed_root():
    """B = 1 (a lone contact, colour 0), 2, 3, 17, 15, 63 bodies; then the
    same with a fixed root."""
    wl = W.custom([1, 1, 1, 1, 3, 1], [1, 2, 3, 17, 5, 63], mu=0.4, controller=W.CTRL_EXTERNAL)
    gs_parity("gs tiny", wl, state_after(wl, 12))
    flags = wl.flags | oracle.FLAG_FIXED_ROOT
    gs_parity("gs fixed root", wl, state_after(wl, 12, flags=flags), flags=flags)


def test_gs_tolerance_stop_counts():
    """Short frictionless chains converge in tens of sweeps; the sweep
    counts of the two precisions agree up to substeps whose residual sits at
    the threshold, and every converged substep ends at or below it."""
    wl = W.custom([1] * 12, [2, 3, 4, 5, 6, 7, 8, 3, 4, 5, 6, 7], controller=W.CTRL_EXTERNAL,
                  tol=1e-4, iters=400, mu=0.0, substeps=1, dt=1 / 240)
    o = oracle.Oracle(wl)
    o.cmd[:] = np.linspace(-1, 1, 12)
    o.run(10)
    oo, g = advance_both(wl, rounded_state(o), **GS)
    print("\n[gs tol] oracle sweeps", oo.iters, "gpu sweeps", g["iters"])
    assert np.all(g["residual"][g["status"] == 0] <= 1e-4)
    assert np.abs(g["iters"] - oo.iters).max() <= 2
    assert (g["iters"] == oo.iters).mean() >= 0.75


def test_gs_graph_equals_direct_and_is_deterministic():
    wl = W.make("uneven", n_snakes=64)
    out = []
    for use_graph in (0, 1, 1):
        sim = snk.Sim(wl, use_graph=use_graph, **GS)
        sim.step(3)
        out.append(sim.read("pos", "quat", "lambda_joint", "lambda_contact", "iters_total"))
        sim.close()
    for r in out[1:]:
        for k in out[0]:
            assert np.array_equal(out[0][k], r[k]), k


def test_gs_serpenoid_and_paper_law_whole_step():
    """The command computed on the device (serpenoid) and the paper's
    pressure law: a whole step gives the oracle's commands and pressures to
    1e-6; the first substep of the step (the law applied once to the held
    command, then one substep) is held to the per-substep gates."""
    from parity import gpu_state, load_gpu

    wl = W.make("uniform", n_snakes=8)
    wl.pressure_law = W.LAW_PAPER
    base = oracle.Oracle(wl)
    base.run(30, threads=8)
    base.commands()
    st = rounded_state(base)
    o = oracle.Oracle(wl, solver=oracle.SOLVER_GS)
    load_oracle(o, st)
    o.step[...] = base.step
    o.run(1, threads=8)
    sim = snk.Sim(wl, **GS)
    load_gpu(sim, st)
    sim.write(step=base.step.copy())
    sim.step(1)
    g = gpu_state(sim)
    cmd = sim.read("cmd")["cmd"]
    sim.close()
    assert np.abs(cmd - o.cmd).max() <= 1e-6
    assert np.abs(g["p"] - o.p).max() <= 1e-6
    oo, g1 = gs_parity("gs paper law first substep", wl, dict(st, cmd=o.cmd.copy()))
    assert np.abs(g1["p"] - oo.p).max() <= 1e-6


def test_gs_full_uniform_batch_sampled():
    """The whole uniform batch in the benchmark's Gauss-Seidel configuration
    (40 sweeps), sampled snakes against the oracle at the per-substep gates
    (the oracle's 1-ulp spread printed as context)."""
    from parity import full_batch_substep

    rng = np.random.default_rng(22)
    pick = sorted({0, 4095, *rng.choice(4096, 6, replace=False).tolist()})
    o, g, sub, st_s, kw = full_batch_substep("uniform", pick, 6, dict(GS, tol=0.0, iters=40),
                                             dict(solver=oracle.SOLVER_GS, tol=0.0, iters=40))
    o2 = oracle.Oracle(sub, **kw)
    load_oracle(o2, dict(st_s, x=np.nextafter(st_s["x"].astype(np.float32), np.float32(np.inf)).astype(np.float64)))
    o2.run(1, threads=8)
    mu = np.asarray(sub.mu, np.float64)
    spread = compare(o, dict(x=o2.x, lam_j=o2.lam_j, lam_c=o2.lam_c), mu)
    err = compare(o, g, mu)
    print("\n[gs full uniform] worst", {k: float(err[k].max()) for k in err if k != "branch"},
          "spread", {k: float(spread[k].max()) for k in ("lam_s", "lam_b", "lam_n", "lam_t")})
    assert np.array_equal(np.asarray(g["iters"]), o.iters)
    assert err["pos"].max() <= POS_TOL
    for k in ("vel", "angvel", "lam_s", "lam_b", "lam_n", "lam_t"):
        assert err[k].max() <= LAM_TOL, k
