"""GPU (FP32 HIP kernels through the C ABI) against the FP64 oracle.

Index work is compared bit for bit.  Physics follows the per-substep
protocol (tests/parity.py): the same FP32-rounded state goes into both, both
take one substep or one step with a fixed iteration count, positions must
agree to 1e-5 relative and multipliers to 1e-4 relative per block type.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import (LAM_TOL, POS_TOL, VEL_TOL, advance_both, compare, f32, gpu_state, load_gpu, load_oracle,
                    rounded_state)

pytestmark = pytest.mark.gpu

snk = pytest.importorskip("paper_1904_02833_amd")


def short_uneven(n, seed=None, max_B=64):
    wl = W.make("uneven", n_snakes=4 * n, seed=seed)
    keep = np.nonzero(wl.bodies <= max_B)[0][:n]
    return wl.take(keep)


def report(tag, err):
    worst = {k: float(np.max(v)) for k, v in err.items()}
    print(f"\n[{tag}] " + " ".join(f"{k}={v:.3g}" for k, v in worst.items()), flush=True)
    return worst


def assert_parity(tag, err, max_branch_frac=0.02, n_bodies=None, lam_tol=LAM_TOL, vel_tol=VEL_TOL):
    worst = report(tag, err)
    assert worst["pos"] <= POS_TOL
    for k in ("lam_s", "lam_b", "lam_n", "lam_t"):
        assert worst[k] <= lam_tol, (k, worst[k])
    for k in ("vel", "angvel"):
        if k in worst:
            assert worst[k] <= vel_tol, (k, worst[k])
    if n_bodies:
        assert err["branch"].sum() <= max_branch_frac * n_bodies


# ---------------------------------------------------------------- index work

@pytest.mark.parametrize("case", ["custom", "uniform", "uneven", "noground"])
def test_index_bit_exact(case):
    if case == "custom":
        wl = W.custom([1, 1, 1, 2, 3, 1, 4, 2, 1], [1, 2, 3, 5, 7, 64, 16, 32, 13])
    elif case == "uniform":
        wl = W.make("uniform", n_snakes=300)
    elif case == "uneven":
        wl = short_uneven(700, max_B=64)
    else:
        wl = W.custom([3, 1, 2], [4, 9, 1], flags=oracle.FLAG_NO_GROUND)
    o = oracle.Oracle(wl)
    ix = o.index()
    sim = snk.Sim(wl)
    for name in snk.INDEX:
        got = sim.index(name)
        want = ix["body_degree" if name == "degree" else name]
        assert got.dtype == np.int32
        assert np.array_equal(got.astype(np.int64), np.asarray(want, np.int64)), name
    sim.close()


# ---------------------------------------------------------------- commands

def test_serpenoid_commands_match():
    wl = W.make("uniform", n_snakes=64)
    sim = snk.Sim(wl)
    o = oracle.Oracle(wl)
    for n in range(5):
        sim.step(1)
        o.commands()
        got = sim.read("cmd")["cmd"]
        assert np.abs(got - o.cmd).max() <= 1e-6
        o.step[:] += 1
    sim.close()


def test_schedule_commands_match():
    wl = short_uneven(120)
    sim = snk.Sim(wl)
    o = oracle.Oracle(wl)
    for n in range(80):
        sim.step(1)
        o.commands()
        assert np.array_equal(sim.read("cmd")["cmd"], o.cmd.astype(np.float32)), n
        o.step[:] += 1
    sim.close()


# ---------------------------------------------------------------- physics

@pytest.mark.parametrize("warm_steps", [1, 40, 200])
def test_substep_parity_single(warm_steps):
    wl = W.make("single")
    o = oracle.Oracle(wl)
    o.run(warm_steps)
    o.commands()
    st = rounded_state(o)
    oo, g = advance_both(wl, st)
    assert_parity(f"single@{warm_steps}", compare(oo, g, wl.mu), n_bodies=64)


def test_step_parity_single():
    """A whole step (4 substeps), substep by substep: the one-launch step
    equals four one-substep launches bit for bit, and each of those is held
    to the per-substep gates against the oracle from the GPU's own state
    before it."""
    from parity import chained_substeps

    wl = W.make("single")
    o = oracle.Oracle(wl)
    o.run(120)
    o.commands()
    for k, (oo, g, _) in enumerate(chained_substeps(wl, rounded_state(o))):
        assert_parity(f"single-step substep {k}", compare(oo, g, wl.mu), n_bodies=64)


def test_substep_parity_uniform_slice():
    wl = W.make("uniform", n_snakes=48)
    o = oracle.Oracle(wl)
    o.run(30, threads=8)
    o.commands()
    oo, g = advance_both(wl, rounded_state(o))
    assert_parity("uniform", compare(oo, g, wl.mu), n_bodies=wl.total_bodies)


def test_substep_parity_uneven_tiles():
    """Snakes of 16..64 bodies: 4, 2 and 1 snakes per wave, ragged tails."""
    wl = short_uneven(150)
    o = oracle.Oracle(wl)
    o.run(25, threads=8)
    o.commands()
    oo, g = advance_both(wl, rounded_state(o))
    assert_parity("uneven", compare(oo, g, wl.mu), n_bodies=wl.total_bodies)


def test_parity_tiny_and_odd_sizes():
    wl = W.custom([1, 1, 1, 1, 3, 1], [1, 2, 3, 17, 5, 63], mu=0.4,
                  controller=W.CTRL_EXTERNAL)
    o = oracle.Oracle(wl)
    o.cmd[:] = np.linspace(-1, 1, o.cmd.size)
    o.run(20)
    oo, g = advance_both(wl, rounded_state(o))
    assert_parity("tiny", compare(oo, g, wl.mu), n_bodies=wl.total_bodies)


@pytest.mark.parametrize("scene", ["cantilever", "resting"])
def test_parity_warm_start_prev(scene):
    """Warm start from the previous substep's multipliers (bodies moved by
    W J^T lambda0 first).  Re-applying unconverged multipliers pumps energy
    into a stiff chain, so the scenes are ones the oracle has settled: a
    cantilever solved to 1e-10 and a chain resting on the ground."""
    if scene == "cantilever":
        wl = W.custom([1], [8], alpha=(1e-3, 2.0, 2.0), controller=W.CTRL_EXTERNAL,
                      flags=oracle.FLAG_FIXED_ROOT | oracle.FLAG_NO_GROUND)
        o = oracle.Oracle(wl, warm=oracle.WARM_PREV, tol=1e-10, iters=200000)
    else:
        wl = W.custom([2], [8], controller=W.CTRL_EXTERNAL)
        o = oracle.Oracle(wl, warm=oracle.WARM_PREV)
    o.run(40)
    assert np.abs(o.v).max() < 1e-6
    oo, g = advance_both(wl, rounded_state(o), warm_start=snk.WARM_PREV)
    assert_parity(f"warm-prev-{scene}", compare(oo, g, wl.mu), n_bodies=16)


def test_parity_warm_start_prev_actuated():
    """The previous-multiplier start on the actuated single snake, where it
    is unstable (its velocities grow about tenfold every ten steps): three
    steps in, while the state is still well scaled, a whole step held to the
    per-substep gates substep by substep from the GPU's own state."""
    from parity import chained_substeps

    wl = W.make("single")
    o = oracle.Oracle(wl, warm=oracle.WARM_PREV)
    o.run(3)
    o.commands()
    for k, (oo, g, _) in enumerate(chained_substeps(wl, rounded_state(o), gpu_over=dict(warm_start=snk.WARM_PREV),
                                                    orc_over=dict(warm=oracle.WARM_PREV))):
        assert_parity(f"warm-prev-actuated substep {k}", compare(oo, g, wl.mu), n_bodies=64)


def test_parity_paper_pressure_law():
    """The paper's pressure law: a whole step gives the oracle's pressures
    to 1e-6; the first substep of a step (the law applied once, then one
    substep, as in the whole step) is held to the per-substep gates."""
    wl = W.make("uniform", n_snakes=8)
    wl.pressure_law = W.LAW_PAPER
    o = oracle.Oracle(wl)
    o.run(30, threads=8)
    o.commands()
    st = rounded_state(o)
    oo, g = advance_both(wl, st, one_substep=False)
    assert np.abs(g["p"] - oo.p).max() <= 1e-6
    oo, g = advance_both(wl, st)
    assert np.abs(g["p"] - oo.p).max() <= 1e-6
    assert_parity("paper-law first substep", compare(oo, g, wl.mu), n_bodies=wl.total_bodies)


def test_parity_cantilever_fixed_root():
    wl = W.custom([1], [12], alpha=(1e-3, 2.0, 2.0), controller=W.CTRL_EXTERNAL,
                  flags=oracle.FLAG_FIXED_ROOT | oracle.FLAG_NO_GROUND)
    o = oracle.Oracle(wl)
    o.run(10)
    oo, g = advance_both(wl, rounded_state(o))
    err = compare(oo, g, wl.mu)
    report("cantilever", err)
    assert err["pos"].max() <= POS_TOL
    assert err["lam_s"].max() <= LAM_TOL and err["lam_b"].max() <= LAM_TOL


def test_trajectory_report_single():
    """Full rollouts drift apart (chaotic contact); reported, not gated,
    beyond staying finite and close for the first steps."""
    wl = W.make("single")
    o = oracle.Oracle(wl)
    sim = snk.Sim(wl)
    errs = []
    for n in range(60):
        o.run(1)
        sim.step(1)
        x = sim.read("pos")["pos"].T
        errs.append(np.abs(x - o.x).max() / np.abs(o.x).max())
    print(f"\n[rollout] pos rel err after 1/10/60 steps: {errs[0]:.2e} {errs[9]:.2e} {errs[-1]:.2e}")
    assert np.all(np.isfinite(errs))
    assert errs[0] <= POS_TOL
    sim.close()


# ---------------------------------------------------------------- runtime

def test_deterministic_and_graph_equals_direct():
    wl = short_uneven(200)
    a = snk.Sim(wl, use_graph=1)
    b = snk.Sim(wl, use_graph=0)
    a.step(7)
    for _ in range(7):
        b.step(1)
    ra, rb = a.read(), b.read()
    for k in ra:
        assert np.array_equal(ra[k], rb[k]), k
    c = snk.Sim(wl, use_graph=1)
    c.step(3)
    c.step(4)
    rc = c.read()
    for k in ra:
        assert np.array_equal(ra[k], rc[k]), k
    for s in (a, b, c):
        s.close()


def test_checkpoint_roundtrip_bitwise():
    wl = W.make("uniform", n_snakes=32)
    a = snk.Sim(wl)
    a.step(10)
    snap = a.read()
    a.step(10)
    end_a = a.read()
    b = snk.Sim(wl)
    b.write(**{k: v for k, v in snap.items()})
    assert all(np.array_equal(b.read()[k], snap[k]) for k in snap)
    b.step(10)
    end_b = b.read()
    for k in end_a:
        assert np.array_equal(end_a[k], end_b[k]), k
    a.close()
    b.close()


def test_nonfinite_snake_is_isolated():
    wl = W.make("uniform", n_snakes=16)
    a = snk.Sim(wl)
    b = snk.Sim(wl)
    a.step(3)
    b.step(3)
    pos = b.read("pos")["pos"]
    pos[0, 64 * 5 + 7] = np.nan          # snake 5, body 7
    b.write(pos=pos)
    a.step(2)
    b.step(2)
    ra, rb = a.read(), b.read()
    assert rb["status"][5] & snk.STATUS_NONFINITE
    others = np.ones(16, bool)
    others[5] = False
    assert np.all(rb["status"][others] == ra["status"][others])
    keep = np.repeat(others, 64)
    assert np.array_equal(ra["pos"][:, keep], rb["pos"][:, keep])
    a.close()
    b.close()


def test_set_pressures_errors_and_device_path():
    import torch
    wl = W.custom([2, 3], 8)
    sim = snk.Sim(wl)
    with pytest.raises(snk.SimError):
        sim.set_pressures(np.array([0.1, np.nan, 0, 0, 0], np.float32))
    with pytest.raises(snk.SimError):
        sim.set_pressures(np.zeros(4, np.float32))
    sim.set_pressures(torch.tensor([2.0, -0.5, float("nan"), 0.25, -3.0], device="cuda"))
    torch.cuda.synchronize()
    assert np.array_equal(sim.read("cmd")["cmd"], np.array([1, -0.5, 0, 0.25, -1], np.float32))
    sim.close()


# ---------------------------------------------------------------- long chains

def test_substep_parity_multiwave_lengths():
    """Snakes spanning 2..16 waves (boundary bodies and residuals through
    LDS), mixed with short ones in the same tiles."""
    wl = W.custom([1, 1, 1, 2, 4, 1, 8, 4, 1, 2], [65, 100, 128, 100, 64, 300, 64, 128, 17, 8],
                  mu=0.5, controller=W.CTRL_EXTERNAL)
    o = oracle.Oracle(wl)
    o.cmd[:] = np.sin(np.arange(o.cmd.size))
    o.run(15, threads=8)
    oo, g = advance_both(wl, rounded_state(o))
    assert_parity("multiwave", compare(oo, g, wl.mu), n_bodies=wl.total_bodies)


def test_substep_parity_uneven_full_range():
    wl = W.make("uneven", n_snakes=90)
    assert wl.bodies.max() > 128
    o = oracle.Oracle(wl)
    o.run(20, threads=8)
    o.commands()
    oo, g = advance_both(wl, rounded_state(o))
    assert_parity("uneven-full", compare(oo, g, wl.mu), n_bodies=wl.total_bodies)


def test_substep_parity_stiff_1024():
    wl = W.make("stiff", n_snakes=2)
    wl.tol, wl.iters = 0.0, 20
    o = oracle.Oracle(wl)
    o.run(6, threads=2)
    o.commands()
    oo, g = advance_both(wl, rounded_state(o))
    assert_parity("stiff", compare(oo, g, wl.mu), n_bodies=wl.total_bodies)


def test_tolerance_mode_matches_oracle_iterations():
    """Tolerance mode on short chains that do converge (several snakes per
    wave stop at different iterations): the iteration counts
    of the two precisions agree up to the substeps whose residual sits at the
    threshold, and every converged substep reports a residual <= tol."""
    # without friction these short chains converge in tens of iterations
    wl = W.custom([1] * 12, [2, 3, 4, 5, 6, 7, 8, 3, 4, 5, 6, 7], controller=W.CTRL_EXTERNAL,
                  tol=1e-4, iters=400, mu=0.0, substeps=1, dt=1 / 240)
    o = oracle.Oracle(wl)
    o.cmd[:] = np.linspace(-1, 1, 12)
    o.run(10)
    st = rounded_state(o)
    oo, g = advance_both(wl, st)
    print("\n[tol] oracle iters", oo.iters, "gpu iters", g["iters"])
    assert np.all(g["residual"][g["status"] == 0] <= 1e-4)
    assert np.abs(g["iters"] - oo.iters).max() <= 2
    assert (g["iters"] == oo.iters).mean() >= 0.75


# ---------------------------------------------------------------- mappings

MAPPINGS = [dict(map_waves=4, map_min_seg=16), dict(map_waves=4, map_min_seg=64),
            dict(map_waves=8, map_min_seg=32), dict(map_waves=16, map_min_seg=16),
            dict(map_waves=4, map_min_seg=16, map_grid=64),
            dict(map_waves=4, map_rows=1), dict(map_waves=16, map_rows=1),
            dict(map_waves=8, map_rows=1, map_grid=64)]


def test_all_mappings_bit_identical():
    wl = W.make("uneven", n_snakes=300)
    ref = None
    for mp in MAPPINGS:
        sim = snk.Sim(wl, **mp)
        sim.step(4)
        r = sim.read()
        print(mp, sim.mapping)
        if ref is None:
            ref = r
        else:
            for k in r:
                assert np.array_equal(r[k], ref[k]), (mp, k)
        sim.close()


def test_autotune_restores_state_and_matches():
    wl = W.make("uneven", n_snakes=200)
    a = snk.Sim(wl, autotune=1)
    b = snk.Sim(wl)
    print("\n[autotune] picked", a.mapping, "default", b.mapping)
    ra0, rb0 = a.read(), b.read()
    for k in ra0:
        assert np.array_equal(ra0[k], rb0[k]), k
    a.step(3)
    b.step(3)
    ra, rb = a.read(), b.read()
    for k in ra:
        assert np.array_equal(ra[k], rb[k]), k
    a.close()
    b.close()


def test_uneven_full_batch_residuals_stay_bounded():
    """The full 16384-snake uneven batch for 30 steps: no snake's residual
    may spike (a spike of |x|/L showed a stale neighbour exchange between
    waves of a spanning snake) and every snake stays finite."""
    wl = W.make("uneven")
    sim = snk.Sim(wl)
    worst = 0.0
    for n in range(30):
        sim.step(1)
        r = sim.read("residual", "status")
        assert not np.any(r["status"] & snk.STATUS_NONFINITE)
        worst = max(worst, float(r["residual"].max()))
        assert r["residual"].max() < 1.0, (n, int(np.argmax(r["residual"])), float(r["residual"].max()))
    print(f"\n[uneven-full] worst residual over 30 steps {worst:.3g}")
    sim.close()


def slice_snakes(st, o_full, sample):
    """Concatenate the per-snake rows of state dict st (whole batch) for the
    sampled snakes, in sample order."""
    out = {}
    for key, off in (("x", o_full.body_off), ("q", o_full.body_off), ("v", o_full.body_off),
                     ("w", o_full.body_off), ("lam_c", o_full.body_off), ("lam_j", o_full.joint_off),
                     ("p", o_full.module_off), ("cmd", o_full.module_off)):
        if key in st:
            out[key] = np.concatenate([st[key][off[s]:off[s + 1]] for s in sample])
    return out


def full_batch_sampled_parity(name, sample, steps=10):
    """The benchmark's settings on a whole named batch: autotuned mapping,
    residual 1e-4 or at most 200 iterations.  The sampled snakes start from
    the oracle's own state after `steps` steps (rounded to FP32), the rest
    of the batch from the GPU's state after the same steps; the whole batch
    takes one more substep on the GPU in the launch configuration the bench
    times, and the sampled snakes take it in the oracle.  Positions 1e-5,
    velocities and multipliers 1e-4, iteration counts equal; the oracle's
    own spread under a one-ulp nudge of its input positions is printed as
    context (the conditioning of the substep), not used as a gate."""
    wl = W.make(name)
    wl.tol, wl.iters = 1e-4, 200
    sample = sorted(sample)
    sub = wl.take(np.array(sample))
    o_lead = oracle.Oracle(sub)
    o_lead.run(steps, threads=8)
    o_lead.commands()
    st_s = rounded_state(o_lead)
    lead = snk.Sim(wl, autotune=1)
    lead.step(steps)
    st = gpu_state(lead)
    lead.close()
    o_full = oracle.Oracle(wl)
    o_full.step[:] = steps
    st["cmd"] = f32(o_full.commands())
    for key, off, soff in (("x", o_full.body_off, o_lead.body_off), ("q", o_full.body_off, o_lead.body_off),
                           ("v", o_full.body_off, o_lead.body_off), ("w", o_full.body_off, o_lead.body_off),
                           ("lam_c", o_full.body_off, o_lead.body_off),
                           ("lam_j", o_full.joint_off, o_lead.joint_off),
                           ("p", o_full.module_off, o_lead.module_off), ("cmd", o_full.module_off, o_lead.module_off)):
        for i, s in enumerate(sample):
            st[key][off[s]:off[s + 1]] = st_s[key][soff[i]:soff[i + 1]]
    h = wl.dt / wl.substeps
    kw = dict(controller=W.CTRL_EXTERNAL, dt=h, substeps=1)
    sim = snk.Sim(wl, autotune=1, **kw)
    load_gpu(sim, st)
    sim.step(1)
    print(f"\n[full-{name}] mapping {sim.mapping}, sampled snakes of {sorted(set(wl.bodies[sample].tolist()))} bodies")
    gs = gpu_state(sim)
    g = slice_snakes(gs, o_full, sample)
    sim.close()
    o = oracle.Oracle(sub, **kw)
    load_oracle(o, st_s)
    o.run(1, threads=8)
    assert np.array_equal(o.iters, gs["iters"][sample])
    o2 = oracle.Oracle(sub, **kw)
    nudged = dict(st_s)
    nudged["x"] = np.nextafter(st_s["x"].astype(np.float32), np.float32(np.inf)).astype(np.float64)
    load_oracle(o2, nudged)
    o2.run(1, threads=8)
    spread = compare(o, dict(x=o2.x, lam_j=o2.lam_j, lam_c=o2.lam_c), sub.mu)
    print(f"[full-{name}] context: FP64 multiplier spread under a 1-ulp input nudge "
          + " ".join(f"{k}={float(np.max(spread[k])):.3g}" for k in ("lam_s", "lam_b", "lam_n", "lam_t")))
    assert_parity(f"full-{name}-sampled", compare(o, g, sub.mu), n_bodies=sub.total_bodies)


def test_full_uniform_batch_sampled_parity():
    """The benchmark's workload in its launch configuration (4096 snakes of
    64 bodies), sampled snakes: first, last, middle and random."""
    rng = np.random.default_rng(11)
    full_batch_sampled_parity("uniform", sorted({0, 1, 2047, 4095, *rng.choice(4096, 8, replace=False).tolist()}))


def test_full_uneven_batch_sampled_parity():
    """The uneven batch (16 384 snakes of 16..256 bodies) in its autotuned
    layout: the longest and shortest snakes, which span waves or share
    them, and random ones."""
    wl = W.make("uneven")
    B = wl.bodies
    rng = np.random.default_rng(12)
    pick = {int(np.argmax(B)), int(np.argmin(B)), 0, wl.n_snakes - 1,
            *np.nonzero(B == 64)[0][:1].tolist(), *rng.choice(wl.n_snakes, 7, replace=False).tolist()}
    full_batch_sampled_parity("uneven", sorted(pick), steps=4)


def test_full_stiff_batch_sampled_parity():
    """The stiff batch (256 snakes of 1024 bodies, 16 waves each)."""
    full_batch_sampled_parity("stiff", [0, 97, 255], steps=3)

def test_rows_layout_on_tiny_and_odd_sizes_bit_identical():
    """Snakes of 1, 2, 3, 15, 17, 63 and 64 bodies in the rows layout (segments
    rounded to 16 lanes, unaligned, crossing waves; with half rows the
    snakes of up to 8 bodies two to a row) give the same bits as the
    aligned layout."""
    wl = W.custom([1, 1, 1, 1, 1, 3, 1, 4] * 20, [1, 2, 3, 15, 17, 5, 63, 16] * 20, mu=0.4)
    ref = None
    for mp in (dict(map_waves=1), dict(map_waves=1, map_rows=1), dict(map_waves=2, map_rows=1),
               dict(map_waves=4, map_rows=1, map_grid=8), dict(map_waves=1, map_rows=2),
               dict(map_waves=2, map_rows=2), dict(map_waves=4, map_rows=2, map_grid=8)):
        sim = snk.Sim(wl, **mp)
        sim.step(6)
        r = sim.read()
        print(mp, sim.mapping)
        if ref is None:
            ref = r
        else:
            for k in r:
                assert np.array_equal(r[k], ref[k]), (mp, k)
        sim.close()


def test_half_rows_on_the_short_batch_bit_identical():
    """The short batch (6 to 8 bodies) with half rows, two snakes to a
    16-lane row (an odd count: the last row holds one snake beside an empty
    half), gives the same bits as with whole rows."""
    wl = W.make("short", n_snakes=301)
    ref = None
    for mp in (dict(map_waves=1, map_rows=1), dict(map_waves=1, map_rows=2), dict(map_waves=4, map_rows=2),
               dict(map_waves=2, map_rows=2, map_grid=16)):
        sim = snk.Sim(wl, **mp)
        sim.step(5)
        r = sim.read()
        print(mp, sim.mapping)
        if ref is None:
            ref = r
        else:
            for k in r:
                assert np.array_equal(r[k], ref[k]), (mp, k)
        sim.close()


def test_zero_iterations_evaluates_only():
    """iters = 0: every substep only evaluates the predicted state; positions
    follow the unconstrained prediction and the residual is that state's."""
    wl = W.make("uneven", n_snakes=60)
    o = oracle.Oracle(wl)
    o.run(10, threads=8)
    o.commands()
    oo, g = advance_both(wl, rounded_state(o), iters=0)
    assert np.all(oo.iters == 0) and np.all(g["iters"] == 0)
    assert_parity("iters0", compare(oo, g, wl.mu), n_bodies=wl.total_bodies)
    rel = np.abs(g["residual"] - oo.residual) / np.maximum(oo.residual, 1e-6)
    assert rel.max() <= 1e-3
