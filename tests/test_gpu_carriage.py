"""GPU parity of the wheeled carriage (section "Rigid Body Joints and
Contact": wheels on hinge joints carry the ground contact) against the FP64
oracle's carriage, both sides in double from the same FP32-rounded state.

They differ by summation order only (the GPU solves its 3x3 blocks by the
adjugate, the oracle by elimination; the GPU sums a body's share of every
block before applying its inverse inertia), and the GPU rounds its result to
the FP32 state arrays (relative 6e-8).  Bound: 1e-6 on segment and wheel
positions and on every multiplier type, each relative to the largest of its
type in the snake (floor: one segment's weight over a substep, m g h^2, and
m g h^2 L for rotational rows); iteration counts and status bits equal.
Lane classes 8 to 1024 (workgroups of 16 waves joined through LDS)."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import f32

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
snk = pytest.importorskip("paper_1904_02833_amd")

TOL = 1e-6
WHEEL_KEYS = ("wx", "wq", "wv", "ww", "lam_w")


def with_wheels(wl):
    wl.flags = wl.flags | oracle.FLAG_WHEELS
    return wl


def carriage(name, n):
    return with_wheels(W.make(name, n_snakes=n))


def state_after(wl, steps, **over):
    o = oracle.Oracle(wl, **over)
    o.run(steps, threads=8)
    o.commands()
    keys = ("x", "q", "v", "w", "p", "cmd", "lam_j") + WHEEL_KEYS
    return {k: f32(getattr(o, k)) for k in keys}


def load_oracle(o, st):
    for k, v in st.items():
        getattr(o, k)[...] = v


def load_gpu(sim, st):
    sim.write(pos=st["x"].T, quat=st["q"].T, vel=st["v"].T, angvel=st["w"].T, pressure=st["p"].T,
              lambda_joint=st["lam_j"].T, wheel_pos=st["wx"].T, wheel_quat=st["wq"].T, wheel_vel=st["wv"].T,
              wheel_angvel=st["ww"].T, lambda_wheel=st["lam_w"].T)
    sim.set_pressures(st["cmd"])


def gpu_state(sim):
    r = sim.read("pos", "quat", "vel", "angvel", "pressure", "lambda_joint", "wheel_pos", "wheel_quat",
                 "wheel_vel", "wheel_angvel", "lambda_wheel", "cmd", "residual", "iters", "status")
    names = dict(x="pos", q="quat", v="vel", w="angvel", p="pressure", lam_j="lambda_joint", wx="wheel_pos",
                 wq="wheel_quat", wv="wheel_vel", ww="wheel_angvel", lam_w="lambda_wheel")
    g = {k: r[v].T.astype(np.float64) for k, v in names.items()}
    g.update(cmd=r["cmd"], residual=r["residual"], iters=r["iters"], status=r["status"])
    return g


def advance_both(wl, st, one_substep=True, **over):
    kw = dict(controller=W.CTRL_EXTERNAL)
    if one_substep:
        kw.update(dt=wl.dt / wl.substeps, substeps=1)
    kw.update(over)
    o = oracle.Oracle(wl, **kw)
    load_oracle(o, st)
    o.run(1, threads=8)
    sim = snk.Sim(wl, **kw)
    load_gpu(sim, st)
    sim.step(1)
    g = gpu_state(sim)
    sim.close()
    return o, g


def errors(o, g):
    """Per-snake worst relative errors by quantity."""
    h = o.batch.dt / o.batch.substeps
    L = o.batch.length
    ref = o.batch.mass * 9.81 * h * h
    cols = {"lam_s": ("lam_j", slice(0, 3), ref), "lam_b": ("lam_j", slice(3, 6), ref * L),
            "lam_h": ("lam_w", slice(0, 3), ref), "lam_a": ("lam_w", [3, 5], ref * L),
            "lam_n": ("lam_w", [6], ref), "lam_t": ("lam_w", [7, 8], ref)}
    out = {k: np.zeros(o.n) for k in ("pos", "wheel_pos", *cols)}
    for s in range(o.n):
        b0, b1 = o.body_off[s], o.body_off[s + 1]
        j0, j1 = o.joint_off[s], o.joint_off[s + 1]
        rows = dict(lam_j=slice(j0, j1), lam_w=slice(2 * b0, 2 * b1))
        out["pos"][s] = np.abs(g["x"][b0:b1] - o.x[b0:b1]).max() / max(np.abs(o.x[b0:b1]).max(), L)
        wo = o.wx[2 * b0:2 * b1]
        out["wheel_pos"][s] = np.abs(g["wx"][2 * b0:2 * b1] - wo).max() / max(np.abs(wo).max(), L)
        for key, (arr, sl, floor) in cols.items():
            lo = getattr(o, arr)[rows[arr]][:, sl]
            lg = g[arr][rows[arr]][:, sl]
            if lo.size:
                out[key][s] = np.abs(lg - lo).max() / max(np.abs(lo).max(), floor)
    return out


def check(o, g, label):
    err = errors(o, g)
    worst = {k: float(v.max()) for k, v in err.items()}
    print(f"\n[{label}] worst {worst}", flush=True)
    assert np.array_equal(np.asarray(g["iters"]), o.iters), "iteration counts differ"
    assert np.array_equal(np.asarray(g["status"]), o.status), "status bits differ"
    for k, v in worst.items():
        assert v <= TOL, k


@pytest.mark.parametrize("name,n,steps", [("short", 48, 8), ("uneven", 24, 8), ("uniform", 12, 8)])
def test_carriage_substep_parity(name, n, steps):
    wl = carriage(name, n)
    st = state_after(wl, steps)
    assert np.abs(st["lam_w"][:, 6]).max() > 0
    o, g = advance_both(wl, st)
    check(o, g, f"carriage substep {name}")


def test_carriage_whole_step_serpenoid_and_paper_law():
    """A whole step (four substeps in one launch, the state in double
    throughout) with the serpenoid command computed on the device and the
    paper's once-per-step pressure law."""
    wl = carriage("uniform", 8)
    wl.pressure_law = W.LAW_PAPER
    base = oracle.Oracle(wl)
    base.run(20, threads=8)
    keys = ("x", "q", "v", "w", "p", "cmd", "lam_j") + WHEEL_KEYS
    st = {k: f32(getattr(base, k)) for k in keys}
    o = oracle.Oracle(wl)
    load_oracle(o, st)
    o.step[...] = base.step
    o.run(1, threads=8)
    sim = snk.Sim(wl)
    load_gpu(sim, st)
    sim.write(step=base.step.copy())
    sim.step(1)
    g = gpu_state(sim)
    sim.close()
    assert np.abs(g["cmd"] - o.cmd).max() <= 1e-6
    assert np.abs(g["p"] - o.p).max() <= 1e-6
    check(o, g, "carriage serpenoid paper law")


def test_carriage_stiff_1024_lanes():
    wl = carriage("stiff", 1)
    st = state_after(wl, 2)
    o, g = advance_both(wl, st)
    check(o, g, "carriage stiff 1024")


def test_carriage_odd_sizes_fixed_root_and_no_ground():
    """B = 1 (one segment on two wheels), 2, 3, 17, 15, 63 and 300 bodies
    (lane classes 8 to 512); the same with a fixed root; and without the
    ground (hinges and joints only)."""
    wl = with_wheels(W.custom([1, 1, 1, 1, 3, 1, 3], [1, 2, 3, 17, 5, 63, 100], mu=0.4,
                              controller=W.CTRL_EXTERNAL))
    rng = np.random.default_rng(3)
    for label, flags in (("odd sizes", wl.flags), ("fixed root", wl.flags | oracle.FLAG_FIXED_ROOT),
                         ("no ground", wl.flags | oracle.FLAG_NO_GROUND)):
        o0 = oracle.Oracle(wl, flags=flags)
        o0.cmd[:] = rng.uniform(-1, 1, o0.cmd.shape)
        o0.run(6)
        keys = ("x", "q", "v", "w", "p", "cmd", "lam_j") + WHEEL_KEYS
        st = {k: f32(getattr(o0, k)) for k in keys}
        o, g = advance_both(wl, st, flags=flags)
        check(o, g, f"carriage {label}")


def test_carriage_tolerance_stop_counts():
    """With a tolerance both sides stop at the same iterate (the rigid
    hinges with sticking wheels converge slowly: thousands of iterations to
    2e-3)."""
    wl = carriage("short", 8)
    st = state_after(wl, 6)
    o, g = advance_both(wl, st, tol=2e-3, iters=20000)
    assert np.all(o.status == 0) and len(set(o.iters.tolist())) > 1
    check(o, g, "carriage tolerance")
    assert np.all(g["residual"] <= 2e-3)


def test_carriage_rolls_and_grips_on_the_gpu():
    """Pushed along its axis the carriage rolls on at the speed that keeps
    each wheel's angular momentum about its contact point; pushed sideways it
    stops (the anisotropic friction of the wheels)."""
    wl = with_wheels(W.custom([1] * 4, [4] * 4, mu=0.5, controller=W.CTRL_EXTERNAL, iters=1000))
    m, R = wl.seg_mass, wl.seg_radius
    mw, rw = m / 8, R / 2
    v0 = 0.02
    sim = snk.Sim(wl)
    r = sim.read("vel", "wheel_vel")
    vel, wvel = r["vel"], r["wheel_vel"]
    vel[0, :8] = wvel[0, :16] = v0      # snakes 0, 1 along x
    vel[1, 8:] = wvel[1, 16:] = v0      # snakes 2, 3 along y
    sim.write(vel=vel, wheel_vel=wvel)
    sim.step(2)
    r = sim.read("vel", "wheel_angvel")
    sim.close()
    M = m + 2 * mw
    v = v0 * M / (M + mw)
    assert np.abs(r["vel"][0, :8] - v).max() <= 1e-3 * v
    assert np.abs(r["wheel_angvel"][1, :16] - v / rw).max() <= 1e-3 * v / rw
    assert np.abs(r["vel"][1, 8:]).max() <= 1e-3 * v0


def test_carriage_graph_equals_direct_and_is_deterministic():
    wl = carriage("uneven", 64)
    out = []
    for use_graph in (0, 1, 1):
        sim = snk.Sim(wl, use_graph=use_graph)
        sim.step(3)
        out.append(sim.read("pos", "quat", "lambda_joint", "wheel_pos", "lambda_wheel", "iters_total"))
        sim.close()
    for r in out[1:]:
        for k in out[0]:
            assert np.array_equal(out[0][k], r[k]), k


def test_carriage_rejects_other_solvers_recording_and_plain_wheel_fields():
    wl = carriage("short", 4)
    for over in (dict(solver=snk.SOLVER_NEWTON), dict(solver=snk.SOLVER_GS), dict(warm_start=snk.WARM_PREV)):
        with pytest.raises(snk.SimError):
            snk.Sim(wl, **over)
    sim = snk.Sim(wl)
    f = torch.empty((1024, 32), device="cuda")
    t = torch.empty((1024, 3), device="cuda")
    with pytest.raises(snk.SimError):
        sim.step_record(1, f, t)
    sim.close()
    plain = snk.Sim(W.make("short", n_snakes=4))
    with pytest.raises(snk.SimError):
        plain.read("wheel_pos")
    plain.close()


def test_carriage_full_uniform_batch_sampled():
    """The whole uniform batch on wheels in the benchmark's configuration
    (4096 snakes, every lane launched), sampled snakes against the oracle."""
    wl = carriage("uniform", 4096)
    rng = np.random.default_rng(23)
    pick = np.array(sorted({0, 4095, *rng.choice(4096, 6, replace=False).tolist()}))
    lead = snk.Sim(wl)
    lead.step(4)
    st_all = gpu_state(lead)
    lead.close()
    o_full = oracle.Oracle(W.make("uniform", n_snakes=4096))
    o_full.step[:] = 4
    st_all["cmd"] = f32(o_full.commands())
    kw = dict(controller=W.CTRL_EXTERNAL, dt=wl.dt / wl.substeps, substeps=1)
    sim = snk.Sim(wl, **kw)
    load_gpu(sim, st_all)
    sim.step(1)
    g_all = gpu_state(sim)
    sim.close()
    B = 64

    def rows(a, per):
        return np.concatenate([a[per * s:per * (s + 1)] for s in pick])

    def sample(st):
        out = {k: rows(st[k], B) for k in ("x", "q", "v", "w")}
        out["lam_j"] = rows(st["lam_j"], B - 1)
        out.update({k: rows(st[k], 4) for k in ("p",)})
        out["cmd"] = rows(st["cmd"], 4)
        out.update({k: rows(st[k], 2 * B) for k in WHEEL_KEYS})
        return out

    sub = wl.take(pick)
    st = sample(st_all)
    g = sample(g_all)
    for k in ("residual", "iters", "status"):
        g[k] = np.asarray(g_all[k])[pick]
    o = oracle.Oracle(sub, **kw)
    load_oracle(o, st)
    o.run(1, threads=8)
    check(o, g, "carriage full uniform")
