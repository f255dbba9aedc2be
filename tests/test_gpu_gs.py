"""GPU block Gauss-Seidel (FP32, colour by colour over the index work's
greedy block colouring) against the FP64 oracle's Gauss-Seidel solver, per
the substep protocol of tests/parity.py: positions to 1e-5, multipliers to
1e-4 relative per block type or the oracle's own FP64 spread under a 1-ulp
input nudge where that is larger, contacts whose active set or stick/slip
branch differs between the precisions counted apart (at most 2 % of
bodies).  Lane classes 8 to 1024."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import LAM_TOL, POS_TOL, advance_both, compare, load_oracle, rounded_state

pytestmark = pytest.mark.gpu
snk = pytest.importorskip("paper_1904_02833_amd")

GS = dict(solver=snk.SOLVER_GS)


def state_after(wl, steps, **over):
    o = oracle.Oracle(wl, **over)
    o.run(steps, threads=8)
    o.commands()
    return rounded_state(o)


def gs_parity(tag, wl, st, one_substep=True, **over):
    """Advance the rounded state st on both sides; multipliers are held per
    type to the larger of 1e-4 and twice the spread of the FP64 oracle's own
    result when its input positions move by one FP32 ulp (the conditioning
    floor of the substep protocol: a Gauss-Seidel solve converges further
    than Jacobi at the same budget, and its converged friction multipliers
    are that sensitive); positions keep 1e-5, sweep counts are equal."""
    o, g = advance_both(wl, st, one_substep=one_substep, **GS, **over)
    kw = dict(controller=W.CTRL_EXTERNAL, solver=oracle.SOLVER_GS, **over)
    if one_substep:
        kw.update(dt=wl.dt / wl.substeps, substeps=1)
    o2 = oracle.Oracle(wl, **kw)
    nudged = dict(st)
    nudged["x"] = np.nextafter(st["x"].astype(np.float32), np.float32(np.inf)).astype(np.float64)
    load_oracle(o2, nudged)
    o2.run(1, threads=8)
    mu = np.asarray(wl.mu, np.float64)
    spread = compare(o, dict(x=o2.x, lam_j=o2.lam_j, lam_c=o2.lam_c), mu)
    err = compare(o, g, mu)
    keys = ("lam_s", "lam_b", "lam_n", "lam_t")
    print(f"\n[{tag}] worst", {k: float(err[k].max()) for k in ("pos",) + keys},
          "FP64 spread", {k: float(spread[k].max()) for k in keys},
          "branch mismatches", int(err["branch"].sum()), flush=True)
    assert np.array_equal(np.asarray(g["iters"]), o.iters)
    assert err["pos"].max() <= POS_TOL
    for k in keys:
        assert err[k].max() <= max(LAM_TOL, 2 * spread[k].max()), k
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
    """A whole step (four substeps, the GPU's state rounded to FP32 between
    them)."""
    wl = W.make("uneven", n_snakes=24)
    gs_parity("gs step uneven", wl, state_after(wl, 10), one_substep=False)


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
    """A whole step with the command computed on the device (serpenoid) and
    the paper's pressure law.  The GPU carries its state in FP32 through the
    four substeps; the multiplier gate is twice the difference between the
    FP64 oracle's step and the same step with its state rounded to FP32
    after every substep (split substeps), or 1e-4 where larger."""
    from parity import f32, gpu_state, load_gpu

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
    r = oracle.Oracle(wl, solver=oracle.SOLVER_GS)
    load_oracle(r, st)
    r.step[...] = base.step
    r.commands()
    for sub in range(wl.substeps):
        for s_ in range(r.n):
            r.solve_substep(s_, r.pre_substep(s_, sub))
        for k in ("x", "q", "v", "w", "lam_j", "lam_c"):
            getattr(r, k)[...] = f32(getattr(r, k))
    sim = snk.Sim(wl, **GS)
    load_gpu(sim, st)
    sim.write(step=base.step.copy())
    sim.step(1)
    g = gpu_state(sim)
    cmd = sim.read("cmd")["cmd"]
    sim.close()
    mu = np.asarray(wl.mu, np.float64)
    spread = compare(o, dict(x=r.x, lam_j=r.lam_j, lam_c=r.lam_c), mu)
    err = compare(o, g, mu)
    print("\n[gs serpenoid paper law] worst", {k: float(err[k].max()) for k in err if k != "branch"},
          "FP32-trajectory spread", {k: float(spread[k].max()) for k in ("lam_s", "lam_b", "lam_n", "lam_t")})
    assert np.abs(cmd - o.cmd).max() <= 1e-6
    assert np.abs(g["p"] - o.p).max() <= 1e-6
    assert np.array_equal(np.asarray(g["iters"]), o.iters)
    assert err["pos"].max() <= POS_TOL
    for k in ("lam_s", "lam_b", "lam_n", "lam_t"):
        assert err[k].max() <= max(LAM_TOL, 2 * spread[k].max()), k


def test_gs_full_uniform_batch_sampled():
    """The whole uniform batch in the benchmark's Gauss-Seidel configuration
    (40 sweeps), sampled snakes against the oracle, with the 1-ulp spread
    gate of the other Gauss-Seidel tests."""
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
    for k in ("lam_s", "lam_b", "lam_n", "lam_t"):
        assert err[k].max() <= max(LAM_TOL, 2 * spread[k].max()), k
