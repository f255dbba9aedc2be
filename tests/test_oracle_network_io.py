"""Pins of the oracle's network inputs and targets (the learned warm start).

The targets are the converged multipliers expressed in the predicted axes of
each joint's first body and divided by a per-type scale; a warm start turns a
prediction back into world multipliers (rotate by that body's predicted
orientation, multiply by the scale) and moves the bodies by W J^T lambda0
before iterating.  The round trip below writes that inverse independently
and holds the oracle's targets to it through the solver: fed back as the
given start, the converged multipliers of a settled chain reproduce its
converged residual at iteration 0.  The multipliers are those of the solve
linearised about the predicted state (Jacobians frozen there), the fixed
point that the one-shot start x <- x~ + W J(x~)^T lambda0 is consistent
with; the nonlinear solve's multipliers differ from them by 1e-4 relative on
this floppy chain, whose iterates swing on the way to convergence.

The input columns are held to closed forms written from their definitions on
a constructed state where every column is non-trivial: a chain of three
modules at a general orientation, off the ground, with distinct pressures,
commands, multipliers and compliances.
"""
import math

import numpy as np

import oracle
import workloads as W
from test_oracle_pins import qmul, rotmat, rotvec_quat

G = 9.81


def settled_cantilever():
    """A six-body cantilever (fixed root, no ground) turned to a general
    orientation and settled under gravity by converged substeps."""
    wl = W.custom([1], [6], alpha=(1e-3, 2.0, 2.0), controller=W.CTRL_EXTERNAL,
                  flags=oracle.FLAG_FIXED_ROOT | oracle.FLAG_NO_GROUND)
    o = oracle.Oracle(wl, tol=1e-12, iters=200000)
    q0 = rotvec_quat(np.array([0.6, -0.35, 0.9]))
    R0 = rotmat(q0)
    o.x[:] = (o.x - o.x[0]) @ R0.T + o.x[0] + np.array([0.0, 0.0, 0.05])
    o.q[:] = np.array([qmul(q0, q) for q in o.q])
    o.run(60)
    assert np.abs(o.v).max() < 1e-6
    return wl, o


def split_state(o):
    return {k: getattr(o, k).copy() for k in ("x", "q", "v", "w", "p", "cmd", "lam_j", "lam_c")}


def load(o, st):
    for k, v in st.items():
        getattr(o, k)[...] = v


def given_start_residual(wl, st, qp, lam_j, **over):
    """Residual of the given start at iteration 0 (no iterations)."""
    o = oracle.Oracle(wl, warm=oracle.WARM_GIVEN, tol=0.0, iters=0, **over)
    load(o, st)
    o.lam_j[...] = lam_j
    o.lam_c[...] = 0.0
    r, it, status = o.solve_substep(0, qp)
    assert it == 0
    return r, o


def test_targets_round_trip_through_the_given_start():
    wl, o = settled_cantilever()
    h = wl.dt / wl.substeps
    ref = wl.seg_mass * G * h * h
    refb = ref * wl.seg_length
    qp = o.pre_substep(0, 0)
    st = split_state(o)
    lin = oracle.Oracle(wl, tol=1e-12, iters=200000, flags=wl.flags | oracle.FLAG_LINEARISED)
    load(lin, st)
    r_star, _, status = lin.solve_substep(0, qp)
    assert status == 0 and r_star <= 1e-12
    lam_star = lin.lam_j.copy()
    tgt = lin.targets(0, qp)
    nj = lam_star.shape[0]
    assert tgt.shape == (2 * nj, 3)
    # the inverse, written from the definition of the targets
    lam0 = np.zeros_like(lam_star)
    for j in range(nj):
        lam0[j, :3] = ref * rotmat(qp[j]) @ tgt[2 * j]
        lam0[j, 3:] = refb * tgt[2 * j + 1]
    assert np.abs(lam0 - lam_star).max() <= 1e-12 * np.abs(lam_star).max()
    r0, og = given_start_residual(wl, st, qp, lam0)
    assert np.array_equal(og.lam_j, lam0)
    rz, _ = given_start_residual(wl, st, qp, np.zeros_like(lam0))
    print(f"\n[targets] residual at iteration 0: given {r0:.3g}, zero {rz:.3g}")
    assert r0 <= 1e-10 and rz >= 1e-3
    # the pin tells the plausible mistakes apart: the transposed rotation
    # and the two scales exchanged each leave a start far from converged
    wrong_rot = lam0.copy()
    wrong_scale = lam0.copy()
    for j in range(nj):
        wrong_rot[j, :3] = ref * rotmat(qp[j]).T @ tgt[2 * j]
        wrong_scale[j, :3] = refb * rotmat(qp[j]) @ tgt[2 * j]
        wrong_scale[j, 3:] = ref * tgt[2 * j + 1]
    for bad in (wrong_rot, wrong_scale):
        rb, _ = given_start_residual(wl, st, qp, bad)
        assert rb >= 1e-3


def test_feature_columns_closed_form():
    """Columns 15-29 and 31 of every joint row, from their definitions:
    chamber pressures of the joint's module after the substep's lag update
    (closed form of the first-order lag), the module's command, the rest
    angle kappa_max (p0 - p1) L inside a module and 0 between modules, the
    block's previous multipliers (stretch in the predicted axes of body A
    over m g h^2; bend-twist over m g h^2 L), log10 of the three scaled
    compliances a / h^2 with a = alpha L, mu, both bodies' previous normal
    multipliers over m g h^2, both predicted heights above contact (z - R) / L,
    and the joint's position j / (B - 1) along the chain."""
    M, S = 3, 4
    alpha = (2e-6, 3e-5, 7e-5)
    mu = 0.37
    wl = W.custom([M], [S], alpha=alpha, mu=mu, controller=W.CTRL_EXTERNAL)
    B = M * S
    o = oracle.Oracle(wl)
    rng = np.random.default_rng(41)
    q0 = rotvec_quat(np.array([0.3, 0.5, -1.1]))
    R0 = rotmat(q0)
    o.x[:] = (o.x - o.x[0]) @ R0.T + np.array([0.0, 0.0, 0.03])
    o.q[:] = np.array([qmul(q0, q) for q in o.q])
    o.v[:] = rng.normal(scale=0.02, size=(B, 3))
    o.w[:] = rng.normal(scale=0.5, size=(B, 3))
    p_start = rng.uniform(0.0, 1.0, size=(M, 2))
    o.p[:] = p_start
    o.cmd[:] = [0.8, -0.6, 0.1]
    o.lam_j[:] = rng.normal(scale=1e-5, size=o.lam_j.shape)
    o.lam_c[:] = np.abs(rng.normal(scale=1e-5, size=o.lam_c.shape))
    lam_j, lam_c = o.lam_j.copy(), o.lam_c.copy()
    x_start, v_start = o.x.copy(), o.v.copy()
    qp = o.pre_substep(0, 0)
    f = o.features(0, qp)
    assert f.shape == (2 * (B - 1), 32)

    h = wl.dt / wl.substeps
    L, R = wl.seg_length, wl.seg_radius
    ref = wl.seg_mass * G * h * h
    # first-order lag toward each chamber's target, one substep
    p_new = np.zeros((M, 2))
    for m in range(M):
        a = o.cmd[m]
        for k, u in enumerate((max(a, 0.0), max(-a, 0.0))):
            tau = wl.tau_inflate if u > p_start[m, k] else wl.tau_deflate
            p_new[m, k] = u + (p_start[m, k] - u) * math.exp(-h / tau)
    z_pred = x_start[:, 2] + h * (v_start[:, 2] - G * h)
    for j in range(B - 1):
        m = j // S
        inside = (j + 1) % S != 0
        theta0 = wl.kappa_max * (p_new[m, 0] - p_new[m, 1]) * L if inside else 0.0
        common = {15: p_new[m, 0], 16: p_new[m, 1], 17: o.cmd[m], 18: theta0,
                  22: math.log10(alpha[0] * L / h ** 2), 23: math.log10(alpha[1] * L / h ** 2),
                  24: math.log10(alpha[2] * L / h ** 2), 25: mu,
                  26: lam_c[j, 0] / ref, 27: lam_c[j + 1, 0] / ref,
                  28: (z_pred[j] - R) / L, 29: (z_pred[j + 1] - R) / L, 31: j / (B - 1)}
        stretch = rotmat(qp[j]).T @ lam_j[j, :3] / ref
        bend = lam_j[j, 3:] / (ref * L)
        for row, prev in ((2 * j, stretch), (2 * j + 1, bend)):
            for col, want in common.items():
                assert abs(f[row, col] - want) <= 1e-12 * max(1.0, abs(want)), (j, row, col)
            assert np.allclose(f[row, 19:22], prev, rtol=1e-12, atol=1e-12 * np.abs(prev).max()), (j, row)
    # the constructed state makes every pinned column vary along the chain
    for col in (15, 16, 17, 18, 19, 20, 21, 26, 27, 28, 29, 31):
        assert np.ptp(f[:, col]) > 0, col
