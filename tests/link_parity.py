"""Helpers of the link solver's GPU-vs-oracle parity tests (the per-substep
protocol of tests/parity.py applied to the full-resolution link): run the
FP64 oracle to a state, round it to FP32, hand the same state to both
sides, advance both by one substep, compare.

Errors per snake:
  pos, frame_pos   max |x_gpu - x_orc| / max(max |x_orc|, link length)
  vel, frame_vel   max |v_gpu - v_orc| / max(max |v_orc|, g h)
  frame_angvel     max |w_gpu - w_orc| / max(max |w_orc|, g h / radius)
  lam_tet, lam_dist, lam_att, lam_n, lam_t
                   max |l_gpu - l_orc| / max(max |l_orc|, floor)
The floor is the multiplier scale of one particle's weight over one substep,
m g h^2 with m the mean particle mass (lam_tet: times the section spacing,
its multipliers being forces times lengths per unit strain); it only
matters where a block type carries no load.  Contacts whose active set or
stick/slip branch differs between the precisions are counted apart and
left out of the contact errors."""
from __future__ import annotations

import numpy as np

import oracle.link as OL
import workloads as W

POS_TOL = 1e-5
LAM_TOL = 1e-4
VEL_TOL = 1e-4
STATE = ("x", "v", "fx", "fq", "fv", "fw", "p", "cmd", "lam_tet", "lam_dist", "lam_att", "lam_c")


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def oracle_state(o: OL.LinkOracle):
    return {k: f32(getattr(o, k)) for k in STATE}


def load_oracle(o: OL.LinkOracle, st):
    for k in STATE:
        getattr(o, k)[...] = st[k]


def load_gpu(sim, st):
    sim.write(pos=st["x"].T, vel=st["v"].T, frame_pos=st["fx"].T, frame_quat=st["fq"].T, frame_vel=st["fv"].T,
              frame_angvel=st["fw"].T, pressure=st["p"].T, lambda_tet=st["lam_tet"].T, lambda_dist=st["lam_dist"],
              lambda_att=st["lam_att"].T, lambda_contact=st["lam_c"].T)
    sim.set_commands(st["cmd"])


def gpu_state(sim):
    r = sim.read()
    out = dict(x=r["pos"].T, v=r["vel"].T, fx=r["frame_pos"].T, fq=r["frame_quat"].T, fv=r["frame_vel"].T,
               fw=r["frame_angvel"].T, p=r["pressure"].T, cmd=r["cmd"], lam_tet=r["lambda_tet"].T,
               lam_dist=r["lambda_dist"], lam_att=r["lambda_att"].T, lam_c=r["lambda_contact"].T)
    out = {k: np.asarray(v, np.float64) for k, v in out.items()}
    out.update(residual=r["residual"], iters=r["iters"], status=r["status"])
    return out


def compare(o: OL.LinkOracle, g: dict):
    """Per-snake error table (dict of arrays) between oracle o and GPU state g."""
    b = o.batch
    n, P, F, T, D, A = o.n, o.P, o.F, o.T, o.D, o.A
    h = b.dt / b.substeps
    m = o.link_masses().mean()
    ref = m * 9.81 * h * h
    sec = b.link_length / (b.sections - 1)
    keys = ("pos", "frame_pos", "frame_quat", "vel", "frame_vel", "frame_angvel", "lam_tet", "lam_dist", "lam_att",
            "lam_n", "lam_t")
    out = {k: np.zeros(n) for k in keys}
    out["branch"] = np.zeros(n, np.int64)
    for s in range(n):
        ps, fs = slice(s * P, (s + 1) * P), slice(s * F, (s + 1) * F)
        xo = o.x[ps]
        out["pos"][s] = np.abs(g["x"][ps] - xo).max() / max(np.abs(xo).max(), b.link_length)
        fo = o.fx[fs]
        out["frame_pos"][s] = np.abs(g["fx"][fs] - fo).max() / max(np.abs(fo).max(), b.link_length)
        qo, qg = o.fq[fs], g["fq"][fs]
        out["frame_quat"][s] = np.minimum(np.abs(qg - qo).max(1), np.abs(qg + qo).max(1)).max()
        vo = o.v[ps]
        out["vel"][s] = np.abs(g["v"][ps] - vo).max() / max(np.abs(vo).max(), 9.81 * h)
        vo = o.fv[fs]
        out["frame_vel"][s] = np.abs(g["fv"][fs] - vo).max() / max(np.abs(vo).max(), 9.81 * h)
        wo = o.fw[fs]
        out["frame_angvel"][s] = np.abs(g["fw"][fs] - wo).max() / max(np.abs(wo).max(), 9.81 * h / b.radius)
        for key, arr, sl, floor in (("lam_tet", "lam_tet", slice(s * T, (s + 1) * T), ref * sec),
                                    ("lam_dist", "lam_dist", slice(s * D, (s + 1) * D), ref),
                                    ("lam_att", "lam_att", slice(s * A, (s + 1) * A), ref)):
            lo = getattr(o, arr)[sl]
            out[key][s] = np.abs(g[arr][sl] - lo).max() / max(np.abs(lo).max(), floor)
        lco, lcg = o.lam_c[ps], g["lam_c"][ps]
        mu = float(o._keep["mu"][s])
        act_o, act_g = lco[:, 0] > 0, lcg[:, 0] > 0
        cap_o = np.linalg.norm(lco[:, 1:], axis=1) >= mu * lco[:, 0] * (1 - 1e-4)
        cap_g = np.linalg.norm(lcg[:, 1:], axis=1) >= mu * lcg[:, 0] * (1 - 1e-4)
        same = (act_o == act_g) & ((cap_o == cap_g) | ~act_o)
        out["branch"][s] = int((~same).sum())
        if same.any():
            sc = max(np.abs(lco[:, 0]).max(), ref)
            out["lam_n"][s] = np.abs(lcg[same, 0] - lco[same, 0]).max() / sc
            out["lam_t"][s] = np.abs(lcg[same, 1:] - lco[same, 1:]).max() / sc
    return out


def advance_both(wl, st, one_substep=True, threads=8, **over):
    """Oracle and GPU from the same FP32 state st, one substep (dt = h,
    substeps = 1) or one step."""
    from paper_1904_02833_amd.link import LinkSim

    kw = dict(over)
    if one_substep:
        kw.update(dt=wl.dt / wl.substeps, substeps=1)
    o = OL.LinkOracle(wl, **kw)
    load_oracle(o, st)
    o.run(1, threads=threads)
    sim = LinkSim(wl, **kw)
    load_gpu(sim, st)
    sim.step(1)
    g = gpu_state(sim)
    sim.close()
    return o, g


def state_after(wl, steps, seed=None, threads=8, **over):
    """The oracle's FP32-rounded state after `steps` steps under the
    workload's drawn commands (the last command held)."""
    o = OL.LinkOracle(wl, **over)
    cmds = W.link_commands(wl, max(steps, 1), seed=seed)
    for n in range(steps):
        o.cmd[:] = cmds[n]
        o.run(1, threads=threads)
    o.cmd[:] = cmds[max(steps - 1, 0)]
    return oracle_state(o)


def report(tag, err):
    worst = {k: float(np.max(v)) for k, v in err.items()}
    print(f"\n[{tag}] " + " ".join(f"{k}={v:.3g}" for k, v in worst.items()), flush=True)
    return worst


def assert_parity(tag, err, n_particles, max_branch_frac=0.02):
    worst = report(tag, err)
    for k in ("pos", "frame_pos"):
        assert worst[k] <= POS_TOL, (k, worst[k])
    assert worst["frame_quat"] <= POS_TOL, worst["frame_quat"]
    for k in ("vel", "frame_vel", "frame_angvel"):
        assert worst[k] <= VEL_TOL, (k, worst[k])
    for k in ("lam_tet", "lam_dist", "lam_att", "lam_n", "lam_t"):
        assert worst[k] <= LAM_TOL, (k, worst[k])
    assert err["branch"].sum() <= max_branch_frac * n_particles


STATE_FIELDS = ("pos", "vel", "frame_pos", "frame_quat", "frame_vel", "frame_angvel", "pressure", "lambda_tet",
                "lambda_dist", "lambda_att", "lambda_contact")


def chained_substeps(wl, st, threads=8, **over):
    """A whole step from st, held to the per-substep protocol substep by
    substep: the GPU takes the step in one launch and again as one launch
    per substep (dt = h, one substep, the same held commands), which must
    give the same bits; each one-substep launch is compared with the
    oracle's substep from the GPU's own FP32 state before it.  Returns the
    (oracle, GPU state) pair of every substep."""
    from paper_1904_02833_amd.link import LinkSim

    whole = LinkSim(wl, **over)
    load_gpu(whole, st)
    whole.step(1)
    g_whole = whole.read(*STATE_FIELDS)
    whole.close()
    one = dict(over, dt=wl.dt / wl.substeps, substeps=1)
    sim = LinkSim(wl, **one)
    load_gpu(sim, st)
    prev, out = st, []
    for _ in range(wl.substeps):
        sim.step(1)
        g = gpu_state(sim)
        o = OL.LinkOracle(wl, **one)
        load_oracle(o, prev)
        o.run(1, threads=threads)
        out.append((o, g))
        prev = {k: g[k] for k in STATE}
    g_chain = sim.read(*STATE_FIELDS)
    sim.close()
    for k in STATE_FIELDS:
        assert np.array_equal(g_whole[k], g_chain[k]), f"one launch and per-substep launches differ in {k}"
    return out
