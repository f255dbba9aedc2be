"""GPU parity of the Newton solver (section "Time-Stepping": Newton
iterations, each solving eq. schur_system with preconditioned
conjugate-residual iterations) against the FP64 oracle's Newton solver.

Both sides compute in double from the same FP32-rounded state and differ
by summation order only; the GPU then rounds its result to its FP32 state
arrays (relative 6e-8).  The bound, 1e-6 on positions and multipliers (in
the parity helpers' relative measures), leaves room for the inner solve to
amplify the summation-order differences a few times.  Lane classes: 8 to
256 lanes (uneven and short batches), 1024 lanes (workgroups of 16 waves
joined through LDS)."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import LAM_TOL, POS_TOL, advance_both, compare, rounded_state

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
snk = pytest.importorskip("paper_1904_02833_amd")

NEWTON = dict(solver=snk.SOLVER_NEWTON, newton_iters=4, pcr_iters=20)
TOL = 1e-6


def state_after(wl, steps, **over):
    o = oracle.Oracle(wl, **over)
    o.run(steps, threads=8)
    o.commands()
    return rounded_state(o)


def check(o, g, wl, label, strict_branch=True):
    err = compare(o, g, np.asarray(wl.mu, np.float64))
    worst = {k: float(err[k].max()) for k in ("pos", "lam_s", "lam_b", "lam_n", "lam_t")}
    print(f"\n[{label}] worst {worst} branch mismatches {int(err['branch'].sum())}")
    assert np.array_equal(np.asarray(g["iters"]), o.iters), "iteration counts differ"
    assert np.array_equal(np.asarray(g["status"]), o.status), "status bits differ"
    for k in ("pos", "lam_s", "lam_b", "lam_n", "lam_t"):
        assert err[k].max() <= TOL, k
    if strict_branch:
        assert err["branch"].sum() == 0


@pytest.mark.parametrize("name,n,steps", [("short", 48, 8), ("uneven", 40, 12), ("uniform", 12, 12)])
def test_newton_substep_parity(name, n, steps):
    wl = W.make(name, n_snakes=n)
    st = state_after(wl, steps)
    o, g = advance_both(wl, st, **NEWTON)
    check(o, g, wl, f"newton substep {name}")


def test_newton_step_parity_uneven():
    """A whole step (four substeps, pressures and commands between them)."""
    wl = W.make("uneven", n_snakes=24)
    st = state_after(wl, 10)
    o, g = advance_both(wl, st, one_substep=False, **NEWTON)
    check(o, g, wl, "newton step uneven")


def test_newton_stiff_1024_lanes():
    wl = W.make("stiff", n_snakes=2)
    st = state_after(wl, 3)
    o, g = advance_both(wl, st, **NEWTON)
    check(o, g, wl, "newton stiff 1024")


def test_newton_tolerance_stop_counts():
    """With a tolerance the solve stops at the first Newton iterate below it;
    both sides stop at the same iterate (same inner-iteration counts)."""
    wl = W.make("short", n_snakes=32)
    flags = wl.flags | oracle.FLAG_NO_GROUND
    st = state_after(wl, 6, flags=flags)
    o, g = advance_both(wl, st, flags=flags, solver=snk.SOLVER_NEWTON, newton_iters=20, pcr_iters=100,
                        tol=1e-7)
    assert np.all(o.status == 0)
    check(o, g, wl, "newton tolerance")
    assert np.all(o.iters < 20 * 100)


def test_newton_fixed_root_and_edge_budgets():
    """Fixed root (infinite mass, contact rows all fixed), a single inner
    iteration, and zero Newton iterations (prediction only)."""
    wl = W.make("short", n_snakes=16)
    flags = wl.flags | oracle.FLAG_FIXED_ROOT
    st = state_after(wl, 5, flags=flags)
    o, g = advance_both(wl, st, flags=flags, **NEWTON)
    check(o, g, wl, "newton fixed root")
    for ni, npc in ((1, 1), (0, 20)):
        o, g = advance_both(wl, st, solver=snk.SOLVER_NEWTON, newton_iters=ni, pcr_iters=npc)
        check(o, g, wl, f"newton {ni}x{npc}")


def test_newton_graph_equals_direct_and_is_deterministic():
    wl = W.make("uneven", n_snakes=64)
    out = []
    for use_graph in (0, 1, 1):
        sim = snk.Sim(wl, use_graph=use_graph, **NEWTON)
        sim.step(3)
        out.append(sim.read("pos", "quat", "lambda_joint", "lambda_contact", "iters_total"))
        sim.close()
    for r in out[1:]:
        for k in out[0]:
            assert np.array_equal(out[0][k], r[k]), k


def test_newton_rejects_recording():
    wl = W.make("short", n_snakes=4)
    sim = snk.Sim(wl, **NEWTON)
    f = torch.empty((1024, 32), device="cuda")
    t = torch.empty((1024, 3), device="cuda")
    with pytest.raises(snk.SimError):
        sim.step_record(1, f, t)
    sim.close()


def test_newton_serpenoid_and_paper_law_whole_steps():
    """A whole step (four substeps in one launch, the state in double
    throughout) with the command computed on the device (serpenoid, phase
    from the step counter) and the paper's once-per-step pressure law."""
    from parity import gpu_state, load_gpu, load_oracle

    wl = W.make("uniform", n_snakes=8)
    wl.pressure_law = W.LAW_PAPER
    base = oracle.Oracle(wl)
    base.run(30, threads=8)
    base.commands()
    st = rounded_state(base)
    o = oracle.Oracle(wl, solver=oracle.SOLVER_NEWTON, newton_iters=4, pcr_iters=20)
    load_oracle(o, st)
    o.step[...] = base.step
    o.run(1, threads=8)
    sim = snk.Sim(wl, **NEWTON)
    load_gpu(sim, st)
    sim.write(step=base.step.copy())
    sim.step(1)
    g = gpu_state(sim)
    cmd = sim.read("cmd")["cmd"]
    sim.close()
    assert np.abs(cmd - o.cmd).max() <= 1e-6
    assert np.abs(g["p"] - o.p).max() <= 1e-6
    check(o, g, wl, "newton serpenoid paper law")


@pytest.mark.parametrize("name", ["uniform", "uneven"])
def test_newton_full_batch_sampled(name):
    """The whole batch in the benchmark's Newton configuration (4 x 20,
    every lane class of the batch launched), sampled snakes against the
    oracle: first, last, the longest and shortest, random ones."""
    from parity import full_batch_substep

    wl = W.make(name)
    rng = np.random.default_rng(21)
    B = wl.bodies
    pick = sorted({0, wl.n_snakes - 1, int(np.argmax(B)), int(np.argmin(B)),
                   *rng.choice(wl.n_snakes, 6, replace=False).tolist()})
    o, g, sub, _, _ = full_batch_substep(name, pick, 6, dict(NEWTON, tol=0.0),
                                         dict(solver=oracle.SOLVER_NEWTON, newton_iters=4, pcr_iters=20, tol=0.0))
    check(o, g, sub, f"newton full {name}")


def test_newton_previous_multiplier_start_substep():
    """The previous substep's multipliers as the start (bodies moved by
    W J(x~)^T lambda0), one substep."""
    wl = W.make("uneven", n_snakes=24)
    st = state_after(wl, 10)
    assert np.abs(st["lam_j"]).max() > 0
    o, g = advance_both(wl, st, warm_start=snk.WARM_PREV, **NEWTON)
    check(o, g, wl, "newton previous start, substep")


def test_newton_previous_multiplier_start_whole_step():
    """A whole step with the previous-multiplier start: each substep starts
    from the last one's multipliers, whose ill-conditioning carries the two
    sides' different summation orders forward over the four substeps, past
    the 1e-6 of the single substeps.  Held to the stated tolerances
    (positions 1e-5, multipliers 1e-4); the oracle's own spread when its
    input positions move by one FP64 ulp is printed as context."""
    from parity import load_oracle

    wl = W.make("uneven", n_snakes=24)
    st = state_after(wl, 10)
    o, g = advance_both(wl, st, one_substep=False, warm_start=snk.WARM_PREV, **NEWTON)
    o2 = oracle.Oracle(wl, controller=W.CTRL_EXTERNAL, solver=oracle.SOLVER_NEWTON, newton_iters=4, pcr_iters=20,
                       warm=oracle.WARM_PREV)
    load_oracle(o2, dict(st, x=np.nextafter(st["x"], np.inf)))
    o2.run(1, threads=8)
    mu = np.asarray(wl.mu, np.float64)
    spread = compare(o, dict(x=o2.x, lam_j=o2.lam_j, lam_c=o2.lam_c), mu)
    err = compare(o, g, mu)
    keys = ("pos", "lam_s", "lam_b", "lam_n", "lam_t")
    print("\n[newton previous start, step] worst", {k: float(err[k].max()) for k in keys},
          "FP64 1-ulp spread", {k: float(spread[k].max()) for k in keys})
    assert np.array_equal(np.asarray(g["iters"]), o.iters)
    assert err["pos"].max() <= POS_TOL
    for k in keys[1:]:
        assert err[k].max() <= LAM_TOL, k


def test_newton_keep_best_matches_oracle():
    """newton_keep_best: each substep ends at its best evaluated Newton
    iterate (kept per lane in LDS), as the oracle's does."""
    wl = W.make("uneven", n_snakes=32)
    st = state_after(wl, 10)
    over = dict(solver=snk.SOLVER_NEWTON, newton_iters=8, pcr_iters=20, newton_keep_best=1)
    o, g = advance_both(wl, st, **over)
    plain, _ = advance_both(wl, st, solver=snk.SOLVER_NEWTON, newton_iters=8, pcr_iters=20)
    assert np.all(o.residual <= plain.residual)
    assert np.any(o.residual < plain.residual)
    check(o, g, wl, "newton keep best")
