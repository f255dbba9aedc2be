"""Shared helpers of the GPU-vs-oracle parity tests (the per-substep
protocol): run the FP64 oracle to a realistic state, round that state to
FP32, hand the same rounded state to both sides, advance both by one
substep (or one step) with the same command, and compare.

Errors reported per snake:
  pos     max |x_gpu - x_orc| / max(max |x_orc|, L)
  vel     max |v_gpu - v_orc| / max(max |v_orc|, g h)        (finalize)
  angvel  max |w_gpu - w_orc| / max(max |w_orc|, g h / L)    (finalize)
  lam_*   max |l_gpu - l_orc| / max(max |l_orc|, l_ref), per block type
The velocity floors are what gravity adds in one substep (g h, and g h / L
for a segment end turning about its centre); they only matter for snakes at
rest.
The floor l_ref is the multiplier scale of one segment's weight over one
substep: m g h^2 (stretch, contact; g = 9.81) and m g h^2 L (bend-twist).
It only matters for snakes whose joints carry almost no load, where the
multipliers are ~1e-9 of that scale and the relative error would divide
rounding noise by ~0.  Contacts whose active set or stick/slip branch differs
between the two precisions are counted separately and left out of the
contact errors."""
from __future__ import annotations

import numpy as np

import oracle
import workloads as W

POS_TOL = 1e-5
LAM_TOL = 1e-4
# velocities come out of the solve like the multipliers (differences of
# positions over one substep), so they take the multipliers' tolerance
VEL_TOL = 1e-4


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def rounded_state(o: oracle.Oracle):
    return dict(x=f32(o.x), q=f32(o.q), v=f32(o.v), w=f32(o.w), p=f32(o.p), cmd=f32(o.cmd),
                lam_j=f32(o.lam_j), lam_c=f32(o.lam_c))


def load_oracle(o: oracle.Oracle, st):
    for k in ("x", "q", "v", "w", "p", "cmd", "lam_j", "lam_c"):
        getattr(o, k)[...] = st[k]


def load_gpu(sim, st):
    sim.write(pos=st["x"].T, quat=st["q"].T, vel=st["v"].T, angvel=st["w"].T,
              pressure=st["p"].T, lambda_joint=st["lam_j"].T, lambda_contact=st["lam_c"].T)
    sim.set_pressures(st["cmd"])


def gpu_state(sim):
    r = sim.read("pos", "quat", "vel", "angvel", "pressure", "lambda_joint", "lambda_contact",
                 "residual", "iters", "status")
    return dict(x=r["pos"].T.astype(np.float64), q=r["quat"].T.astype(np.float64),
                v=r["vel"].T.astype(np.float64), w=r["angvel"].T.astype(np.float64),
                p=r["pressure"].T.astype(np.float64), lam_j=r["lambda_joint"].T.astype(np.float64),
                lam_c=r["lambda_contact"].T.astype(np.float64), residual=r["residual"],
                iters=r["iters"], status=r["status"])


def compare(o: oracle.Oracle, g: dict, mu):
    """Per-snake error table (dict of arrays) between oracle o and GPU state g."""
    n = o.n
    vel = "v" in g and "w" in g
    keys = ("pos", "vel", "angvel", "lam_s", "lam_b", "lam_n", "lam_t") if vel else \
        ("pos", "lam_s", "lam_b", "lam_n", "lam_t")
    out = {k: np.zeros(n) for k in keys}
    out["branch"] = np.zeros(n, np.int64)
    L = o.batch.length
    h = o.batch.dt / o.batch.substeps
    ref = o.batch.mass * 9.81 * h * h
    floor = {"lam_s": ref, "lam_b": ref * L}
    for s in range(n):
        b0, b1 = o.body_off[s], o.body_off[s + 1]
        j0, j1 = o.joint_off[s], o.joint_off[s + 1]
        xo, xg = o.x[b0:b1], g["x"][b0:b1]
        out["pos"][s] = np.abs(xg - xo).max() / max(np.abs(xo).max(), L)
        if vel:
            vo, vg = o.v[b0:b1], g["v"][b0:b1]
            out["vel"][s] = np.abs(vg - vo).max() / max(np.abs(vo).max(), 9.81 * h)
            wo, wg = o.w[b0:b1], g["w"][b0:b1]
            out["angvel"][s] = np.abs(wg - wo).max() / max(np.abs(wo).max(), 9.81 * h / L)
        for key, sl in (("lam_s", slice(0, 3)), ("lam_b", slice(3, 6))):
            lo, lg = o.lam_j[j0:j1, sl], g["lam_j"][j0:j1, sl]
            if lo.size:
                out[key][s] = np.abs(lg - lo).max() / max(np.abs(lo).max(), floor[key])
        lco, lcg = o.lam_c[b0:b1], g["lam_c"][b0:b1]
        act_o, act_g = lco[:, 0] > 0, lcg[:, 0] > 0
        cap_o = np.linalg.norm(lco[:, 1:], axis=1) >= mu[s] * lco[:, 0] * (1 - 1e-4)
        cap_g = np.linalg.norm(lcg[:, 1:], axis=1) >= mu[s] * lcg[:, 0] * (1 - 1e-4)
        same = (act_o == act_g) & ((cap_o == cap_g) | ~act_o)
        out["branch"][s] = int((~same).sum())
        if same.any():
            sc = max(np.abs(lco[:, 0]).max(), ref)
            out["lam_n"][s] = np.abs(lcg[same, 0] - lco[same, 0]).max() / sc
            out["lam_t"][s] = np.abs(lcg[same, 1:] - lco[same, 1:]).max() / sc
    return out


def advance_both(wl, st, one_substep=True, threads=8, **over):
    """Build an oracle and a GPU sim for `wl` (external commands), load the
    rounded state st into both, advance one substep (or one step)."""
    import paper_1904_02833_amd as snk

    kw = dict(controller=W.CTRL_EXTERNAL)
    if one_substep:
        kw.update(dt=wl.dt / wl.substeps, substeps=1)
    kw.update(over)
    o = oracle.Oracle(wl, **{k: v for k, v in kw.items() if k not in ("warm_start", "use_graph")},
                      warm=kw.get("warm_start", 0))
    load_oracle(o, st)
    o.run(1, threads=threads)
    sim = snk.Sim(wl, **kw)
    load_gpu(sim, st)
    sim.step(1)
    g = gpu_state(sim)
    sim.close()
    return o, g


def slice_rows(st, o_full, sample):
    """Concatenate the per-snake rows of state dict st (whole batch) for the
    sampled snakes, in sample order."""
    out = {}
    for key, off in (("x", o_full.body_off), ("q", o_full.body_off), ("v", o_full.body_off),
                     ("w", o_full.body_off), ("lam_c", o_full.body_off), ("lam_j", o_full.joint_off),
                     ("p", o_full.module_off), ("cmd", o_full.module_off)):
        if key in st:
            out[key] = np.concatenate([st[key][off[s]:off[s + 1]] for s in sample])
    return out


def full_batch_substep(name, sample, steps, gpu_over, orc_over):
    """A whole named batch on the GPU: `steps` plain steps, then one substep
    of the whole batch with the solver settings gpu_over; the sampled snakes
    take the same substep in the oracle (settings orc_over) from the same
    FP32 state and commands.  Returns the oracle of the sample, the GPU
    state of the sample, the sampled workload, the sampled FP32 state and
    the oracle keyword arguments of the substep."""
    import paper_1904_02833_amd as snk

    wl = W.make(name)
    lead = snk.Sim(wl)
    lead.step(steps)
    st = gpu_state(lead)
    lead.close()
    o_full = oracle.Oracle(wl)
    o_full.step[:] = steps
    st["cmd"] = f32(o_full.commands())
    kw = dict(controller=W.CTRL_EXTERNAL, dt=wl.dt / wl.substeps, substeps=1)
    sim = snk.Sim(wl, **kw, **gpu_over)
    load_gpu(sim, st)
    sim.step(1)
    g_all = gpu_state(sim)
    sim.close()
    g = slice_rows(g_all, o_full, sample)
    for k in ("residual", "iters", "status"):
        g[k] = np.asarray(g_all[k])[sample]
    sub = wl.take(np.array(sample))
    st_s = slice_rows(st, o_full, sample)
    o = oracle.Oracle(sub, **kw, **orc_over)
    load_oracle(o, st_s)
    o.run(1, threads=8)
    return o, g, sub, st_s, dict(kw, **orc_over)


STATE_FIELDS = ("pos", "quat", "vel", "angvel", "pressure", "lambda_joint", "lambda_contact")


def chained_substeps(wl, st, gpu_over=None, orc_over=None, threads=8):
    """A whole step from the rounded state st, held to the per-substep
    protocol substep by substep.  The GPU takes the step once in a single
    launch (all substeps, state in registers throughout) and once as one
    launch per substep (dt = h, one substep, the same held command); the
    two must give the same bits.  Each one-substep launch is then compared
    with the oracle's substep from the same FP32 state, the GPU's own state
    before it, so an error does not compound across substeps.  Returns the
    (oracle, GPU state, FP32 state before the substep) of every substep.  The lag law only: the
    paper's law acts once per step, which one-substep launches cannot
    reproduce."""
    import paper_1904_02833_amd as snk

    assert wl.pressure_law == W.LAW_LAG
    gpu_over = dict(gpu_over or {})
    orc_over = dict(orc_over or {})
    base = dict(controller=W.CTRL_EXTERNAL)
    whole = snk.Sim(wl, **base, **gpu_over)
    load_gpu(whole, st)
    whole.step(1)
    g_whole = whole.read(*STATE_FIELDS)
    whole.close()
    one = dict(base, dt=wl.dt / wl.substeps, substeps=1)
    sim = snk.Sim(wl, **one, **gpu_over)
    load_gpu(sim, st)
    prev, out = st, []
    for _ in range(wl.substeps):
        sim.step(1)
        g = gpu_state(sim)
        o = oracle.Oracle(wl, **one, **orc_over)
        load_oracle(o, prev)
        o.run(1, threads=threads)
        out.append((o, g, prev))
        prev = dict(x=g["x"], q=g["q"], v=g["v"], w=g["w"], p=g["p"], cmd=st["cmd"], lam_j=g["lam_j"],
                    lam_c=g["lam_c"])
    g_chain = sim.read(*STATE_FIELDS)
    sim.close()
    for k in STATE_FIELDS:
        assert np.array_equal(g_whole[k], g_chain[k]), f"one launch and per-substep launches differ in {k}"
    return out
