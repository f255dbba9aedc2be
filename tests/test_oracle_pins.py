"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
formulas: they check closed forms, invariants, limits, symmetries, finite
differences and a dense direct solve of the linearised compliant system
(eq. schur_system).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

H60 = 1.0 / 60.0


def chain(M, S, **kw):
    return W.custom(M, S, **kw)


def quat_about_z(phi):
    return np.array([math.cos(phi / 2), 0.0, 0.0, math.sin(phi / 2)])


def qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def rotvec_quat(v):
    th = np.linalg.norm(v)
    if th == 0:
        return np.array([1.0, 0, 0, 0])
    return np.concatenate([[math.cos(th / 2)], math.sin(th / 2) * v / th])


def rotmat(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


# ---------------------------------------------------------------- pressure

def test_lag_closed_form():
    """First-order lag: p(t) = u + (p0 - u) exp(-t/tau) at every step
    boundary, tau_inflate while rising and tau_deflate while falling."""
    wl = chain(1, 4, controller=W.CTRL_EXTERNAL, flags=oracle.FLAG_NO_GROUND, gravity=0.0)
    o = oracle.Oracle(wl)
    o.cmd[:] = 0.8
    for n in range(1, 31):
        o.run(1)
        t = n * H60
        assert abs(o.p[0, 0] - 0.8 * (1 - math.exp(-t / 0.1))) < 1e-14
        assert o.p[0, 1] == 0.0
    p0 = o.p[0, 0]
    o.cmd[:] = -0.3          # chamber 0 vents toward 0, chamber 1 inflates to 0.3
    for n in range(1, 31):
        o.run(1)
        t = n * H60
        assert abs(o.p[0, 0] - p0 * math.exp(-t / 0.2)) < 1e-14
        assert abs(o.p[0, 1] - 0.3 * (1 - math.exp(-t / 0.1))) < 1e-14


def test_lag_substep_invariance():
    """The lag is the exact solution for a held target, so the pressure at a
    step boundary does not depend on the number of substeps."""
    res = []
    for sub in (1, 3, 8):
        wl = chain(1, 2, controller=W.CTRL_EXTERNAL, flags=oracle.FLAG_NO_GROUND, gravity=0.0,
                   substeps=sub)
        o = oracle.Oracle(wl)
        o.cmd[:] = 0.65
        o.run(7)
        res.append(o.p[0, 0])
    assert max(res) - min(res) < 1e-15


def test_paper_law_inflation_and_deflation():
    """eq. delta_p_i / eq. deflation with k_i = k_d = 0.23, T_p = 0.68 psi
    (fitted values of the step-response experiment), p_s = A = 8 psi.
    Inflation from 0 to the full source pressure: the first step adds
    k_i p_s; the remaining error e obeys 1/e_{n+1} - 1/e_n -> k_i/p_s.
    Deflation from 8 psi: linear 0.68 psi per step while k_d p > T_p, then
    geometric with ratio 1 - k_d."""
    wl = chain(1, 2, controller=W.CTRL_EXTERNAL, flags=oracle.FLAG_NO_GROUND, gravity=0.0,
               pressure_law=W.LAW_PAPER)
    o = oracle.Oracle(wl)
    o.cmd[:] = 1.0
    psi = []
    for _ in range(400):
        o.run(1)
        psi.append(o.p[0, 0] * 8.0)
    psi = np.array(psi)
    assert abs(psi[0] - 0.23 * 8.0) < 1e-13
    assert np.all(np.diff(psi) > 0) and np.all(psi < 8.0)
    e = 8.0 - psi
    slope = 1 / e[-1] - 1 / e[-2]
    assert abs(slope - 0.23 / 8.0) < 1e-4
    # deflation
    o.p[0, 0] = 1.0
    o.cmd[:] = 0.0
    psi = [8.0]
    for _ in range(40):
        o.run(1)
        psi.append(o.p[0, 0] * 8.0)
    psi = np.array(psi)
    thresh = 0.68 / 0.23
    for n in range(1, len(psi)):
        prev = psi[n - 1]
        want = prev - 0.68 if prev * 0.23 > 0.68 else prev * (1 - 0.23)
        assert abs(psi[n] - want) < 1e-12
    assert psi[8] < thresh < psi[7]      # 8 - 0.68 n crosses 2.957 between n = 7 and 8
    assert abs(psi[8] - (8 - 8 * 0.68)) < 1e-12
    assert abs(psi[12] - (8 - 8 * 0.68) * 0.77 ** 4) < 1e-12


# ---------------------------------------------------------------- command

def test_serpenoid_values():
    """eq. snake_control: at f = 0.25 Hz, t = 1 s the sine argument of
    module m is pi/2 + m pi/2, so the commands are 1, 0, -1, 0; an offset
    of 0.5 clamps at 1."""
    wl = chain(4, 2, controller=W.CTRL_SERPENOID, freq=0.25, phase0=0.0)
    o = oracle.Oracle(wl)
    o.step[:] = 59
    o.commands()
    assert np.allclose(o.cmd, [1, 0, -1, 0], atol=1e-15)
    o2 = oracle.Oracle(wl, ctrl_offset=0.5)
    o2.step[:] = 59
    o2.commands()
    assert np.allclose(o2.cmd, [1, 0.5, -0.5, 0.5], atol=1e-15)


def test_schedule_pieces():
    wl = chain(1, 2, controller=W.CTRL_SCHEDULE)
    wl.sched_off = np.array([0, 2], np.int32)
    wl.sched_steps = np.array([3, 2], np.int32)
    wl.sched_val = np.array([0.2, 0.7])
    o = oracle.Oracle(wl, flags=oracle.FLAG_NO_GROUND)
    seen = []
    for n in range(7):
        o.step[:] = n
        seen.append(o.commands()[0])
    assert seen == [0.2, 0.2, 0.2, 0.7, 0.7, 0.7, 0.7]


# ---------------------------------------------------------------- geometry

def arc_state(B, theta0, L=0.01):
    """Closed-form chain on its rest arc: body j turned by j theta0 about z,
    neighbouring end points coincident (centres on a regular polygon with
    side L cos(theta0/2))."""
    x = np.zeros((B, 3))
    q = np.zeros((B, 4))
    for j in range(B):
        phi = j * theta0
        q[j] = quat_about_z(phi)
        if j:
            a0 = np.array([math.cos((j - 1) * theta0), math.sin((j - 1) * theta0), 0])
            a1 = np.array([math.cos(phi), math.sin(phi), 0])
            x[j] = x[j - 1] + 0.5 * L * (a0 + a1)
    return x, q


def test_free_arc_is_a_fixed_point():
    """Zero gravity, no ground, held pressure: a chain placed on the closed
    form arc of its rest shape stays there.  Pins the rest-angle sign
    (positive command bends toward +z rotation) and the stretch/bend forms."""
    M, S = 1, 12
    wl = chain(M, S, controller=W.CTRL_EXTERNAL, gravity=0.0, flags=oracle.FLAG_NO_GROUND)
    o = oracle.Oracle(wl)
    o.p[:] = [[0.6, 0.0]]
    o.cmd[:] = 0.6
    theta0 = 10.0 * 0.6 * 0.01
    x, q = arc_state(M * S, theta0)
    o.x[:] = x
    o.q[:] = q
    o.run(50)
    assert np.abs(o.x - x).max() < 1e-12
    assert np.abs(o.q - q).max() < 1e-12
    assert o.residual[0] < 1e-12


def shape_invariants(x, q):
    rel = [qmul(np.array([q[j][0], *-q[j][1:]]), q[j + 1]) for j in range(len(q) - 1)]
    ang = np.array([2 * math.atan2(r[3], r[0]) for r in rel])
    dist = np.linalg.norm(np.diff(x, axis=0), axis=1)
    return ang, dist


def test_straight_chain_converges_to_arc():
    """Started straight, the free chain settles on the rest arc (shape
    invariants: relative turn theta0 per joint, centre spacing L cos(theta0/2))."""
    wl = chain(2, 4, controller=W.CTRL_EXTERNAL, gravity=0.0, flags=oracle.FLAG_NO_GROUND,
               alpha=(1e-4, 1e-4, 1e-4))
    o = oracle.Oracle(wl, tol=1e-13, iters=100000)
    o.cmd[:] = [0.5, -0.25]
    o.run(600)
    ang, dist = shape_invariants(o.x, o.q)
    p0, p1 = o.p[0, 0], o.p[1, 1]
    th = np.array([10 * p0 * 0.01] * 3 + [0.0] + [-10 * p1 * 0.01] * 3)
    assert abs(p0 - 0.5) < 1e-12 and abs(p1 - 0.25) < 1e-12
    assert np.abs(ang - th).max() < 1e-9
    assert np.abs(dist - 0.01 * np.cos(th / 2)).max() < 1e-11


def test_rest_without_gravity_is_exact():
    """A straight chain at rest, no pressure, no gravity stays exactly put."""
    wl = chain(4, 16, controller=W.CTRL_EXTERNAL, gravity=0.0)
    o = oracle.Oracle(wl)
    x0 = o.x.copy()
    o.run(600)
    assert np.abs(o.x - x0).max() <= 1e-14
    assert np.abs(o.v).max() <= 1e-14


def test_rest_on_ground_settles():
    """On the ground under gravity a straight unactuated chain sinks to a
    steady penetration and comes to rest: its velocity decays, it does not
    creep, nothing drives it sideways, and the penetration stays below a few
    g h^2 (the part of each substep's fall the fixed iterations leave)."""
    wl = chain(4, 16, controller=W.CTRL_EXTERNAL)
    o = oracle.Oracle(wl)
    x0 = o.x.copy()
    o.run(300)
    x300 = o.x.copy()
    o.run(300)
    assert np.abs(o.v).max() < 1e-9
    assert np.abs(o.x[:, 1]).max() == 0.0
    # the unconverged iterations leave the ends slightly curled; the
    # second-order asymmetry of the bend linearisation then creeps the chain
    # by ~1e-11 m per step, far below anything visible at 1 cm bodies
    assert np.abs(o.x - x300).max() < 1e-8
    assert np.abs(o.x[:, 0] - x0[:, 0]).max() < 1e-7
    pen = 0.01 - o.x[:, 2]
    assert 0 < pen.max() < 9.81 * (1 / 240) ** 2 * 5


def test_initial_residual_closed_form():
    """With zero iterations nothing is corrected: the chain falls freely, the
    reported residual is the contact violation alone.  After substep k of
    implicit Euler from rest the drop is g h^2 k (k+1)/2, so over 4 substeps
    the step's largest residual is 10 g h^2 / L (1 g h^2 / L for one)."""
    h = H60 / 4
    for sub, tri in ((4, 10), (1, 1)):
        wl = chain(2, 8, controller=W.CTRL_EXTERNAL, substeps=sub, dt=h * sub)
        o = oracle.Oracle(wl, iters=0)
        o.run(1)
        assert abs(o.residual[0] - tri * 9.81 * h * h / 0.01) < 1e-14
        assert o.iters[0] == 0


# ---------------------------------------------------------------- Jacobian

def perturbed_chain(B, rng, amp=2e-3, rot=0.2):
    x = np.zeros((B, 3))
    q = np.zeros((B, 4))
    for i in range(B):
        x[i] = [(i + 0.5) * 0.01, 0.0, 0.01]
        x[i] += rng.normal(scale=amp, size=3)
        q[i] = rotvec_quat(rng.normal(scale=rot, size=3))
    return x, q


@pytest.mark.parametrize("B", [2, 3, 5])
def test_jacobian_matches_finite_differences(B):
    """Every Jacobian column equals the central difference of the
    constraint vector; rotations are perturbed by exact world-frame turns."""
    rng = np.random.default_rng(7 + B)
    wl = chain(1, B)
    o = oracle.Oracle(wl)
    x, q = perturbed_chain(B, rng)
    xp = x - rng.normal(scale=1e-3, size=x.shape)
    p = np.array([[0.4, 0.1]])
    C0, J, Wm, comp = o.assemble(0, x, q, xp, p)
    eps = 1e-6
    for i in range(B):
        for d in range(6):
            xa, xb, qa, qb = x.copy(), x.copy(), q.copy(), q.copy()
            if d < 3:
                xa[i, d] += eps
                xb[i, d] -= eps
            else:
                e = np.zeros(3)
                e[d - 3] = eps
                qa[i] = qmul(rotvec_quat(e), q[i])
                qb[i] = qmul(rotvec_quat(-e), q[i])
            Ca = o.assemble(0, xa, qa, xp, p)[0]
            Cb = o.assemble(0, xb, qb, xp, p)[0]
            fd = (Ca - Cb) / (2 * eps)
            assert np.allclose(J[:, 6 * i + d], fd, rtol=1e-6, atol=1e-8), (i, d)


def test_inverse_mass_blocks():
    """Rotation block of W is the inverse of the world inertia of a solid
    cylinder along the body x axis: eigenvalues 1/I_axis and 1/I_perp, the
    1/I_axis eigenvector being the rotated body x axis."""
    rng = np.random.default_rng(3)
    wl = chain(1, 2)
    o = oracle.Oracle(wl)
    x, q = perturbed_chain(2, rng)
    _, _, Wm, _ = o.assemble(0, x, q, x, np.zeros((1, 2)))
    m, R, L = 0.02, 0.01, 0.01
    Iax, Ipe = m * R * R / 2, m * (3 * R * R + L * L) / 12
    for i in range(2):
        assert np.allclose(Wm[6 * i:6 * i + 3, 6 * i:6 * i + 3], np.eye(3) / m)
        Wr = Wm[6 * i + 3:6 * i + 6, 6 * i + 3:6 * i + 6]
        ev = np.sort(np.linalg.eigvalsh(Wr))
        assert np.allclose(ev, np.sort([1 / Iax, 1 / Ipe, 1 / Ipe]), rtol=1e-12)
        axis = rotmat(q[i]) @ np.array([1.0, 0, 0])
        assert np.allclose(Wr @ axis, axis / Iax, rtol=1e-10)


# ---------------------------------------------------------------- KKT

@pytest.mark.parametrize("B,ground", [(2, False), (3, False), (4, False), (2, True), (3, True), (4, True)])
def test_linearised_jacobi_matches_dense_kkt(B, ground):
    """Tiny chains: the linearised block-Jacobi iteration (Jacobians frozen at
    the predicted state) converges to the solution of
    (J W J^T + E/h^2) lambda = -C(x~), the compliant system of
    eq. schur_system, solved densely.  With ground every contact is pressed
    in and mu is large, so every contact row is an active equality."""
    rng = np.random.default_rng(100 * B + ground)
    flags = oracle.FLAG_LINEARISED | (0 if ground else oracle.FLAG_NO_GROUND)
    wl = chain(1, B, controller=W.CTRL_EXTERNAL, alpha=(3e-4, 2e-3, 1e-3), mu=1e6,
               substeps=1, dt=1 / 240)
    o = oracle.Oracle(wl, flags=flags, tol=1e-13, iters=2_000_000)
    x0, q0 = perturbed_chain(B, rng, amp=1e-4, rot=0.02 if ground else 0.2)
    v0 = rng.normal(scale=0.05, size=(B, 3))
    w0 = rng.normal(scale=1.0, size=(B, 3))
    if ground:
        x0[:, 2] = 0.01 - 3e-3
        v0[:, 2] = -0.5
        w0 *= 0.1
    o.x[:], o.q[:], o.v[:], o.w[:] = x0, q0, v0, w0
    o.p[:] = [[0.3, 0.0]]
    o.cmd[:] = 0.3
    # predicted state, computed by the oracle's own stage on a copy
    ref = oracle.Oracle(wl, flags=flags)
    ref.x[:], ref.q[:], ref.v[:], ref.w[:] = x0, q0, v0, w0
    d = ref.predict(0, 1 / 240)
    Cv, J, Wm, comp = o.assemble(0, d["x"], d["q"], x0, o.p)
    A = J @ Wm @ J.T + np.diag(comp)
    lam_dense = np.linalg.solve(A, -Cv)
    if ground:   # premise: every contact is pressed in at the solution
        assert np.all(lam_dense[6 * (B - 1)::3] > 0)
    o.run(1)
    assert o.status[0] == 0, o.residual
    lam = np.concatenate([o.lam_j.reshape(-1), o.lam_c.reshape(-1) if ground else []])
    scale = np.abs(lam_dense).max()
    assert np.abs(lam - lam_dense).max() <= 1e-10 * scale
    if ground:
        assert np.all(o.lam_c[:, 0] > 0)


@pytest.mark.parametrize("B,ground", [(3, False), (5, False), (3, True), (5, True)])
def test_first_jacobi_iterations_in_closed_form(B, ground):
    """The linearised iteration is scaled block Jacobi on the compliant
    system A lambda = -C (A = J W J^T + E/h^2, eq. schur_system):
    lambda_{k+1} = lambda_k - S D^{-1} (C + A lambda_k), D the 3x3 diagonal
    blocks of A and S the per-block factor 1 / (most blocks on one of its
    bodies).  Checked for the first three iterations from lambda = 0, with
    D and S built here from the dense matrix and the chain's structure."""
    rng = np.random.default_rng(5 * B + ground)
    flags = oracle.FLAG_LINEARISED | (0 if ground else oracle.FLAG_NO_GROUND)
    wl = chain(1, B, controller=W.CTRL_EXTERNAL, alpha=(3e-4, 2e-3, 1e-3), mu=1e6,
               substeps=1, dt=1 / 240)
    x0, q0 = perturbed_chain(B, rng, amp=1e-4, rot=0.02)
    v0 = rng.normal(scale=0.05, size=(B, 3))
    if ground:
        x0[:, 2] = 0.01 - 3e-3
        v0[:, 2] = -0.5
    ref = oracle.Oracle(wl, flags=flags)
    ref.x[:], ref.q[:], ref.v[:] = x0, q0, v0
    d = ref.predict(0, 1 / 240)
    Cv, J, Wm, comp = ref.assemble(0, d["x"], d["q"], x0, np.zeros((1, 2)))
    A = J @ Wm @ J.T + np.diag(comp)
    nb = len(Cv) // 3
    deg = [(1 if ground else 0) + 2 * (i > 0) + 2 * (i < B - 1) for i in range(B)]
    scale = [1 / max(deg[j], deg[j + 1]) for j in range(B - 1) for _ in (0, 1)]
    scale += [1 / deg[i] for i in range(B)] if ground else []
    lam = np.zeros(len(Cv))
    for k in range(1, 4):
        r = Cv + A @ lam
        step = np.zeros_like(lam)
        for n in range(nb):
            sl = slice(3 * n, 3 * n + 3)
            step[sl] = -scale[n] * np.linalg.solve(A[sl, sl], r[sl])
        lam = lam + step
        o = oracle.Oracle(wl, flags=flags, iters=k)
        o.x[:], o.q[:], o.v[:] = x0, q0, v0
        o.run(1)
        got = np.concatenate([o.lam_j.reshape(-1), o.lam_c.reshape(-1) if ground else []])
        assert np.abs(got - lam).max() <= 1e-11 * np.abs(lam).max(), k


def test_twist_spring_single_substep():
    """Body 0 clamped, body 1 spinning slowly about the chain axis (which
    leaves the shared end point in place, so only the twist row acts).  One
    converged implicit substep of a torsion spring of compliance a_t and
    axial inertia I_x gives twist h w0 / (1 + h^2 / (a_t I_x)) (linear regime);
    the bend compliance, ten times larger, must not enter."""
    h, w0 = 1 / 240, 1e-3
    a_t, a_b = 5.0, 50.0
    wl = chain(1, 2, controller=W.CTRL_EXTERNAL, alpha=(1e-3, a_b, a_t), gravity=0.0,
               substeps=1, dt=h)
    o = oracle.Oracle(wl, flags=oracle.FLAG_FIXED_ROOT | oracle.FLAG_NO_GROUND, tol=1e-15,
                      iters=100000)
    o.w[1] = [w0, 0, 0]
    o.run(1)
    twist = 2 * math.atan2(o.q[1, 1], o.q[1, 0])
    Ix = 0.5 * 0.02 * 0.01 ** 2
    want = h * w0 / (1 + h * h / (a_t * 0.01 * Ix))
    assert abs(twist - want) < 1e-6 * abs(want)


# ---------------------------------------------------------------- statics

def cantilever(B, a_s, a_b, substeps=4):
    """Clamped chain; each substep starts from the previous multipliers
    (the warm start moves the bodies by W J^T lambda0 before iterating)."""
    wl = chain(1, B, controller=W.CTRL_EXTERNAL, alpha=(a_s, a_b, a_b), substeps=substeps)
    return oracle.Oracle(wl, flags=oracle.FLAG_FIXED_ROOT | oracle.FLAG_NO_GROUND,
                         tol=1e-12, iters=200000, warm=oracle.WARM_PREV)


def cantilever_closed_form(B, a_s, a_b, m=0.02, g=9.81, L=0.01):
    """Small-deflection statics of a chain clamped at body 0: joint j at
    p_j = (j+1) L carries shear V_j and moment M_j of all bodies beyond it;
    joint j turns by a_b M_j and shears by a_s V_j (a = per-length value * L)."""
    xs = (np.arange(B) + 0.5) * L
    pj = (np.arange(B - 1) + 1.0) * L
    V = np.array([g * m * (B - 1 - j) for j in range(B - 1)])
    Mo = np.array([g * m * sum(xs[k] - pj[j] for k in range(j + 1, B)) for j in range(B - 1)])
    defl = np.zeros(B)
    for k in range(1, B):
        defl[k] = sum(a_b * L * Mo[j] * (xs[k] - pj[j]) + a_s * L * V[j] for j in range(k))
    return defl


def test_cantilever_closed_form():
    """Compliant cantilever chain under gravity: settled deflections match
    the small-deflection closed form; at delta/l ~ 1e-3 the geometric
    non-linearity leaves a relative difference of order 1e-5."""
    B = 6
    a_s, a_b = 1e-3, 2.0
    o = cantilever(B, a_s, a_b)
    o.run(300)
    assert np.abs(o.v).max() < 1e-10
    want = cantilever_closed_form(B, a_s, a_b)
    got = 0.01 - o.x[:, 2]
    assert want[-1] / (B * 0.01) < 2e-3
    assert np.abs(got[1:] - want[1:]).max() <= 2e-5 * want[-1]


def test_compliance_to_zero_limit():
    """As the compliance goes to 0 the converged residual goes to 0 and the
    stretch violation divided by the compliance tends to the static joint
    force (the weight carried beyond the joint)."""
    B = 3
    ratios = []
    for a in (1e-2, 1e-4, 1e-6):
        o = cantilever(B, a, a)
        o.run(200)
        assert o.residual[0] <= 1e-12
        d = o.snake(0)
        x, q = d["x"], d["q"]
        # stretch violation of joint 0 from the end points
        r0 = rotmat(q[0]) @ [0.005, 0, 0]
        r1 = rotmat(q[1]) @ [-0.005, 0, 0]
        Cs = (x[0] + r0) - (x[1] + r1)
        ratios.append(np.linalg.norm(Cs) / (a * 0.01))
    force = 9.81 * 0.02 * (B - 1)
    for r in ratios:
        assert abs(r - force) < 1e-6 * force


# ---------------------------------------------------------------- friction

@pytest.mark.parametrize("v0,iters", [(0.3, 20), (0.02, 20), (0.3, 1)])
def test_single_body_sliding_stop(v0, iters):
    """One body sliding on the ground: each substep the Coulomb cone caps
    the slip correction at mu g h^2, so v drops by mu g h per substep and
    stops exactly once it falls below mu g h.  A single body touches one
    block, so one iteration already gives this: the tangential projection
    uses the normal multiplier of the same iteration."""
    mu, h = 0.5, 1 / 240
    wl = chain(1, 1, controller=W.CTRL_EXTERNAL, mu=mu, substeps=1, dt=h, iters=iters)
    o = oracle.Oracle(wl)
    o.v[0] = [v0, 0, 0]
    v = v0
    for n in range(40):
        o.run(1)
        v = v - mu * 9.81 * h if v > mu * 9.81 * h else 0.0
        assert abs(o.v[0, 0] - v) < 1e-12
        assert abs(o.v[0, 2]) < 1e-12
    assert o.v[0, 0] == 0.0


def test_friction_and_quaternion_invariants():
    """Along a driven run: lambda_n >= 0, |lambda_t| <= mu lambda_n and
    |q| = 1 (the cone and the unit-quaternion state of the paper)."""
    wl = W.make("single")
    o = oracle.Oracle(wl)
    for _ in range(60):
        o.run(1)
        ln = o.lam_c[:, 0]
        lt = np.linalg.norm(o.lam_c[:, 1:], axis=1)
        assert np.all(ln >= 0)
        assert np.all(lt <= 0.5 * ln * (1 + 1e-12) + 1e-300)
        assert np.abs(np.linalg.norm(o.q, axis=1) - 1).max() < 1e-12


# ---------------------------------------------------------------- conservation

def test_linear_momentum_conserved_without_external_forces():
    """Zero gravity and no ground: internal constraint impulses come in equal
    and opposite pairs, so the total linear momentum is conserved."""
    rng = np.random.default_rng(11)
    wl = chain(3, 5, controller=W.CTRL_EXTERNAL, gravity=0.0, flags=oracle.FLAG_NO_GROUND)
    o = oracle.Oracle(wl)
    o.v[:] = rng.normal(scale=0.1, size=o.v.shape)
    o.w[:] = rng.normal(scale=2.0, size=o.w.shape)
    P0 = o.v.sum(0)
    for n in range(50):
        o.cmd[:] = np.sin(0.3 * n + np.arange(3))
        o.run(1)
        assert np.abs(o.v.sum(0) - P0).max() < 1e-12


def test_free_spin_decay_closed_form():
    """A free body spinning about its symmetry axis: the gyroscopic torque
    vanishes, and the first-order quaternion update turns it by
    2 atan(h w / 2) per substep, so the recovered rate is
    w / sqrt(1 + (h w / 2)^2)."""
    h = 1 / 240
    wl = chain(1, 1, controller=W.CTRL_EXTERNAL, gravity=0.0, flags=oracle.FLAG_NO_GROUND,
               substeps=1, dt=h)
    o = oracle.Oracle(wl)
    w = 30.0
    o.w[0] = [w, 0, 0]
    for _ in range(20):
        o.run(1)
        w = w / math.sqrt(1 + (h * w / 2) ** 2)
        assert abs(o.w[0, 0] - w) < 1e-9
        assert np.abs(o.w[0, 1:]).max() < 1e-12


def test_gyroscopic_term_conserves_angular_momentum():
    """Torque-free tumbling of the cylinder: one substep changes the world
    angular momentum I_w w only at second order in h (halving h quarters
    the change); a wrong sign of the gyroscopic torque would make it first
    order and about 0.15 h |w| in size."""
    m, R, L = 0.02, 0.01, 0.01
    Ib = np.diag([m * R * R / 2, m * (3 * R * R + L * L) / 12, m * (3 * R * R + L * L) / 12])

    def drift(h):
        wl = chain(1, 1, controller=W.CTRL_EXTERNAL, gravity=0.0, flags=oracle.FLAG_NO_GROUND,
                   substeps=1, dt=h)
        o = oracle.Oracle(wl)
        o.w[0] = [20.0, 15.0, 0.0]

        def Lw():
            Rm = rotmat(o.q[0])
            return Rm @ Ib @ Rm.T @ o.w[0]

        L0 = Lw()
        o.run(1)
        return np.linalg.norm(Lw() - L0) / np.linalg.norm(L0)

    h = 1 / 2400
    d1, d2 = drift(h), drift(h / 2)
    assert d1 < 0.05 * h * 25.0
    assert d1 / d2 > 3.5


# ---------------------------------------------------------------- symmetry

def test_mirror_symmetry():
    """Negating every command swaps the chambers and mirrors the motion in
    the x-z plane: y -> -y, q -> (w, -x, y, -z)."""
    wl = chain(3, 6, controller=W.CTRL_EXTERNAL, mu=0.4)
    a = oracle.Oracle(wl)
    b = oracle.Oracle(wl)
    for n in range(120):
        c = np.sin(2 * math.pi * 0.7 * (n + 1) / 60 + np.arange(3) * math.pi / 2)
        a.cmd[:] = c
        b.cmd[:] = -c
        a.run(1)
        b.run(1)
    assert np.abs(a.x[:, 1]).max() > 1e-5
    assert np.abs(a.x[:, [0, 2]] - b.x[:, [0, 2]]).max() < 1e-12
    assert np.abs(a.x[:, 1] + b.x[:, 1]).max() < 1e-12
    assert np.abs(a.q * [1, -1, 1, -1] - b.q).max() < 1e-12
    assert np.abs(a.p[:, ::-1] - b.p).max() == 0.0


# ---------------------------------------------------------------- index work

def test_colouring_closed_form_and_offsets():
    """Sequential greedy colouring in block-list order (joints as
    stretch_j, bend_j, then contacts) on a chain: stretch_j -> 2 (j mod 2),
    bend_j -> 2 (j mod 2) + 1, first contact 2, interior contacts 4, last
    contact 2 if B-2 is even else 0; B = 2 gives 2, 2; B = 1 gives 0."""
    Ms = np.array([1, 1, 1, 2, 3, 1, 4, 2], np.int32)
    Ss = np.array([1, 2, 3, 5, 7, 64, 16, 32], np.int32)
    wl = chain(Ms, Ss)
    o = oracle.Oracle(wl)
    ix = o.index()
    Bs = Ms.astype(int) * Ss
    assert list(ix["body_off"]) == [0] + list(np.cumsum(Bs))
    assert list(ix["joint_off"]) == [0] + list(np.cumsum(Bs - 1))
    assert list(ix["module_off"]) == [0] + list(np.cumsum(Ms))
    for s, B in enumerate(Bs):
        b0 = ix["block_off"][s]
        col = ix["blk_color"][b0:ix["block_off"][s + 1]]
        want = []
        for j in range(B - 1):
            want += [2 * (j % 2), 2 * (j % 2) + 1]
        for i in range(B):
            if B == 1:
                want.append(0)
            elif B == 2:
                want.append(2)
            elif i == 0:
                want.append(2)
            elif i == B - 1:
                want.append(2 if (B - 2) % 2 == 0 else 0)
            else:
                want.append(4)
        assert list(col) == want, B
        deg = ix["body_degree"][ix["body_off"][s]:ix["body_off"][s + 1]]
        if B == 1:
            assert list(deg) == [1]
        else:
            assert deg[0] == deg[-1] == 3 and np.all(deg[1:-1] == 5)
        assert ix["bucket"][s] == (int(B) - 1).bit_length()
    order = np.lexsort((np.arange(len(Bs)), -Bs))
    assert list(ix["order"]) == list(order)


# ---------------------------------------------------------------- split substep

def test_split_substeps_equal_whole_step():
    """Prediction and solve run separately give the whole step bit for bit."""
    wl = W.make("single")
    a = oracle.Oracle(wl)
    a.run(30)
    b = oracle.Oracle(wl, controller=W.CTRL_EXTERNAL)
    for k in ("x", "q", "v", "w", "p", "lam_j", "lam_c"):
        getattr(b, k)[...] = getattr(a, k)
    a.commands()
    b.cmd[:] = a.cmd
    a.run(1)
    for sub in range(4):
        qp = b.pre_substep(0, sub)
        b.solve_substep(0, qp)
    for k in ("x", "q", "v", "w", "p", "lam_j", "lam_c"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k


def test_fallback_keeps_better_start_and_rejects_worse():
    """A given start equal to the zero-start solution's multipliers begins
    closer and is kept; a wild start begins farther, falls back, and then
    reproduces the zero-start substep exactly."""
    wl = W.custom([2], [6], controller=W.CTRL_EXTERNAL, substeps=1, dt=1 / 240)
    base = oracle.Oracle(wl)
    base.cmd[:] = [0.5, -0.5]
    base.run(5)
    st = {k: getattr(base, k).copy() for k in ("x", "q", "v", "w", "p", "cmd", "lam_j", "lam_c")}

    def run(warm, lam_j=None, lam_c=None):
        o = oracle.Oracle(wl, warm=warm, fallback=1)
        for k, vv in st.items():
            getattr(o, k)[...] = vv
        qp = o.pre_substep(0, 0)
        if lam_j is not None:
            o.lam_j[...] = lam_j
            o.lam_c[...] = lam_c
        r = o.solve_substep(0, qp)
        return o, r

    z, rz = run(oracle.WARM_ZERO)
    good, rg = run(oracle.WARM_GIVEN, z.lam_j, z.lam_c)
    assert not (rg[2] & oracle.STATUS_FELL_BACK if hasattr(oracle, "STATUS_FELL_BACK") else rg[2] & 4)
    assert rg[0] < rz[0]
    bad, rb = run(oracle.WARM_GIVEN, np.full_like(z.lam_j, 1e-3), np.full_like(z.lam_c, 1e-3))
    assert rb[2] & 4
    assert np.array_equal(bad.x, z.x) and np.array_equal(bad.lam_j, z.lam_j)


def test_features_closed_form_and_yaw_invariance():
    """Straight chain at rest after the prediction: every constraint value
    and relative velocity vanishes, gravity points along body z, and the
    penetration feature is -g h^2 / L; turning the whole chain about the
    vertical leaves every feature unchanged."""
    wl = W.custom([2], [5], controller=W.CTRL_EXTERNAL)
    o = oracle.Oracle(wl)
    o.cmd[:] = 0.0
    qp = o.pre_substep(0, 0)
    f = o.features(0, qp)
    h = 1 / 240
    assert f.shape == (18, 32)
    assert np.abs(f[:, 0:12]).max() < 1e-13
    assert np.allclose(f[:, 12:15], [0, 0, 1], atol=1e-15)
    assert np.allclose(f[:, 28:30], -9.81 * h * h / 0.01, rtol=1e-12)
    assert np.array_equal(f[0::2, 30], np.zeros(9)) and np.array_equal(f[1::2, 30], np.ones(9))
    # a bent, moving chain, then the same turned by 0.7 rad about z
    rng = np.random.default_rng(2)
    o2 = oracle.Oracle(wl)
    o2.cmd[:] = [0.7, -0.3]
    o2.run(20)
    o2.v[:] += rng.normal(scale=0.01, size=o2.v.shape)
    o2.w[:] += rng.normal(scale=0.3, size=o2.w.shape)
    o3 = oracle.Oracle(wl)
    yaw = rotvec_quat(np.array([0, 0, 0.7]))
    Rz = rotmat(yaw)
    o3.x[:] = o2.x @ Rz.T
    o3.v[:] = o2.v @ Rz.T
    o3.w[:] = o2.w @ Rz.T
    o3.q[:] = np.array([qmul(yaw, q) for q in o2.q])
    for k in ("p", "cmd", "lam_c"):
        getattr(o3, k)[...] = getattr(o2, k)
    o3.lam_j[:, :3] = o2.lam_j[:, :3] @ Rz.T
    o3.lam_j[:, 3:] = o2.lam_j[:, 3:]
    f2 = o2.features(0, o2.pre_substep(0, 0))
    f3 = o3.features(0, o3.pre_substep(0, 0))
    assert np.abs(f2 - f3).max() < 1e-10


def test_fallback_after_k_iterations_follows_the_probes():
    """With fallback_k = K the start is chosen by the residuals after K
    iterations from each start (computed here by separate runs), and the
    substep then equals the chosen start's plain solve (continued from its
    iterate K), with the other start's K iterations counted on top."""
    K, iters = 4, 25
    wl = W.custom([2], [6], controller=W.CTRL_EXTERNAL, substeps=1, dt=1 / 240)
    base = oracle.Oracle(wl)
    base.cmd[:] = [0.5, -0.5]
    base.run(5)
    st = {k: getattr(base, k).copy() for k in ("x", "q", "v", "w", "p", "cmd", "lam_j", "lam_c")}

    def run(warm, n, lam=None, **kw):
        o = oracle.Oracle(wl, warm=warm, iters=n, tol=0.0, **kw)
        for k, vv in st.items():
            getattr(o, k)[...] = vv
        qp = o.pre_substep(0, 0)
        if lam is not None:
            o.lam_j[...] = lam[0]
            o.lam_c[...] = lam[1]
        r = o.solve_substep(0, qp)
        return o, r

    zero_long, _ = run(oracle.WARM_ZERO, 200)
    starts = {"good": (zero_long.lam_j.copy(), zero_long.lam_c.copy()),
              "wild": (np.full_like(zero_long.lam_j, 1e-3), np.full_like(zero_long.lam_c, 1e-3))}
    kept = set()
    for name, lam in starts.items():
        _, rz = run(oracle.WARM_ZERO, K)
        _, rw = run(oracle.WARM_GIVEN, K, lam)
        o, r = run(oracle.WARM_GIVEN, iters, lam, fallback=1, fallback_k=K)
        if rw[0] <= rz[0]:
            ref, rr = run(oracle.WARM_GIVEN, iters, lam)
            assert not (r[2] & 4) and r[1] == iters + K
            kept.add(name)
        else:
            ref, rr = run(oracle.WARM_ZERO, iters)
            assert (r[2] & 4) and r[1] == iters + K
        for k in ("x", "q", "lam_j", "lam_c"):
            assert np.array_equal(getattr(o, k), getattr(ref, k)), (name, k)
        assert r[0] == rr[0]
    assert kept == {"good"}


def test_previous_multiplier_start_diverges_on_the_actuated_chain():
    """Re-applying the previous substep's unconverged multipliers as
    displacements pumps energy into the actuated 64-body snake: with the
    paper's 4 x 20 budget its largest speed grows by orders of magnitude in
    30 steps, while the zero start stays at centimetres per second."""
    wl = W.make("single")
    speed = {}
    for warm in (oracle.WARM_ZERO, oracle.WARM_PREV):
        o = oracle.Oracle(wl, warm=warm)
        o.run(30)
        speed[warm] = float(np.abs(o.v).max())
    assert speed[oracle.WARM_ZERO] < 0.05
    assert speed[oracle.WARM_PREV] > 100.0
