"""Pins of the oracle's wheel carriage (section "Rigid Body Joints and
Contact": rigid wheels on hinge joints carry the ground contact, Coulomb
friction at the wheel's contact point; section "Soft robotic snake model":
the wheels give the snake its anisotropic friction).

Pinned by: the weight a resting carriage puts on its wheels (total normal
multiplier = total mass x g x h^2 per substep); rolling against sliding (a
carriage pushed along its axis rolls on at the speed that conserves each
wheel's angular momentum about its contact point, with spin v / r, one
pushed sideways stops); the Jacobians of every block type against central
finite differences of the constraint values; and the converged block-Jacobi
solve against a dense direct solve of the linearised system."""
import numpy as np
import pytest

import oracle
import workloads as W


def carriage(n_modules=(2,), segs=(4,), **kw):
    wl = W.custom(list(n_modules), list(segs), mu=0.5, controller=W.CTRL_EXTERNAL, **kw)
    wl.flags = wl.flags | oracle.FLAG_WHEELS
    return wl


def test_resting_carriage_puts_its_weight_on_the_wheels():
    wl = carriage()
    o = oracle.Oracle(wl, tol=1e-10, iters=5000)
    x0, wx0 = o.x.copy(), o.wx.copy()
    o.run(3)
    B = int(o.B[0])
    h = wl.dt / wl.substeps
    m, mw = wl.seg_mass, wl.seg_mass / 8
    total = B * (m + 2 * mw) * wl.gravity * h * h
    assert abs(o.lam_w[:, 6].sum() - total) <= 1e-9 * total
    assert np.all(o.lam_w[:, 6] > 0)
    assert np.abs(o.x - x0).max() <= 1e-9 and np.abs(o.wx - wx0).max() <= 1e-9
    # the wheels sit on the ground, centre at height r = R/2
    assert np.abs(o.wx[:, 2] - wl.seg_radius / 2).max() <= 1e-9


def test_rolling_keeps_its_closed_form_speed_and_sliding_stops():
    """Pushed along its axis at v0 the carriage rolls on at
    v0 M / (M + sum I_axle / r^2) (mass M; each wheel's angular momentum
    about its contact point is conserved as it starts to roll), wheels
    spinning at v / r (to 1e-4: the first-order step loses a few 1e-5 of
    the rolling speed per step; a wheel's axial inertia taken as m r^2 / 4
    would be off by 5 %); pushed sideways at v0 it stops."""
    wl = carriage(n_modules=(1,), segs=(4,))
    m, R = wl.seg_mass, wl.seg_radius
    mw, rw = m / 8, R / 2
    v0 = 0.02
    o = oracle.Oracle(wl, tol=1e-11, iters=100000)
    o.v[:, 0] = v0
    o.wv[:, 0] = v0
    o.run(2)
    B = int(o.B[0])
    M = B * (m + 2 * mw)
    v = v0 * M / (M + 2 * B * 0.5 * mw * rw * rw / (rw * rw))
    assert abs(o.v[:, 0].mean() - v) <= 1e-4 * v
    assert np.abs(o.wv[:, 0] - v).max() <= 1e-4 * v
    # spin about the axle (world y at rest): omega = v / r
    assert np.abs(o.ww[:, 1] - v / rw).max() <= 1e-4 * v / rw
    s = oracle.Oracle(wl, tol=1e-11, iters=100000)
    s.v[:, 1] = v0
    s.wv[:, 1] = v0
    s.run(2)
    assert np.abs(s.v[:, 1]).max() <= 1e-6 * v0
    assert np.abs(s.ww).max() <= 1e-6 * v0 / rw


def rotate(q, th):
    """q <- exp(th) q for a world rotation vector th (exact)."""
    a = np.linalg.norm(th)
    if a == 0:
        return q.copy()
    ax = th / a
    r = np.r_[np.cos(a / 2), np.sin(a / 2) * ax]
    w1, x1, y1, z1 = r
    w2, x2, y2, z2 = q
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def random_pose(rng, B, R, L):
    """Segments near a straight chain, wheels near their hinge points,
    everything turned by a few degrees."""
    n = 3 * B
    x = np.zeros((n, 3))
    x[:B, 0] = (np.arange(B) + 0.5) * L
    x[:B, 2] = R
    for i in range(B):
        for k in range(2):
            x[B + 2 * i + k] = x[i] + [0, R if k == 0 else -R, -R / 2]
    x += rng.normal(0, 0.1 * R, x.shape)
    q = np.zeros((n, 4))
    for b in range(n):
        q[b] = rotate(np.array([1.0, 0, 0, 0]), rng.normal(0, 0.15, 3))
    return x, q


def test_wheel_block_jacobians_match_finite_differences():
    wl = carriage(n_modules=(1,), segs=(3,))
    o = oracle.Oracle(wl)
    B = int(o.B[0])
    rng = np.random.default_rng(5)
    xp, qp = random_pose(rng, B, wl.seg_radius, wl.seg_length)
    x, q = xp + rng.normal(0, 1e-3, xp.shape), np.array([rotate(a, rng.normal(0, 0.05, 3)) for a in qp])
    p = np.array([[0.3, 0.0]])
    Cv, J, _, _ = o.assemble_wheels(0, x, q, xp, qp, p)
    eps = 1e-6
    Jfd = np.zeros_like(J)
    for b in range(3 * B):
        for d in range(6):
            xs, qs = [x.copy(), x.copy()], [q.copy(), q.copy()]
            for sgn, k in ((1, 0), (-1, 1)):
                if d < 3:
                    xs[k][b, d] += sgn * eps
                else:
                    e = np.zeros(3)
                    e[d - 3] = sgn * eps
                    qs[k][b] = rotate(q[b], e)
            cp = o.assemble_wheels(0, xs[0], qs[0], xp, qp, p)[0]
            cm = o.assemble_wheels(0, xs[1], qs[1], xp, qp, p)[0]
            Jfd[:, 6 * b + d] = (cp - cm) / (2 * eps)
    assert np.abs(J - Jfd).max() <= 1e-6 * max(1.0, np.abs(J).max())
    # the hinge axis block's spin row carries nothing
    nj = 2 * (B - 1)
    for wi in range(2 * B):
        r = 3 * (nj + 3 * wi + 1) + 1
        assert Cv[r] == 0 and not J[r].any()


def test_linearised_solve_meets_the_dense_solve_without_ground():
    """Linearised, no ground: block-Jacobi run to 1e-13 reaches
    dl = A^-1 (-C), A = J W J^T + diag(alpha~) over the joint and hinge rows
    (the spin rows dropped), assembled at the predicted state."""
    wl = carriage(n_modules=(1,), segs=(3,), substeps=1)
    flags = wl.flags | oracle.FLAG_NO_GROUND | oracle.FLAG_LINEARISED
    o = oracle.Oracle(wl, flags=flags, tol=1e-13, iters=400000)
    o.cmd[...] = 0.5
    o.run(2)
    st = {k: getattr(o, k).copy() for k in ("x", "q", "v", "w", "wx", "wq", "wv", "ww", "p")}
    o.run(1)
    B = int(o.B[0])
    assert o.status[0] == 0
    xs, qs = np.r_[st["x"], st["wx"]], np.r_[st["q"], st["wq"]]
    vs, ws = np.r_[st["v"], st["wv"]], np.r_[st["w"], st["ww"]]
    xt, qt, _, _ = o.predict_bodies(0, xs, qs, vs, ws, wl.dt)
    Cv, J, Wm, comp = o.assemble_wheels(0, xt, qt, xs, qs, o.p)
    nj = 2 * (B - 1)
    keep = [r for r in range(len(Cv)) if not (r // 3 >= nj and (r // 3 - nj) % 2 == 1 and r % 3 == 1)]
    Cv, J, comp = Cv[keep], J[keep], comp[keep]
    dl = np.linalg.solve(J @ Wm @ J.T + np.diag(comp), -Cv)
    got = np.r_[o.lam_j.reshape(-1), o.lam_w[:, [0, 1, 2, 3, 5]].reshape(-1)]
    assert np.abs(got - dl).max() <= 1e-8 * np.abs(dl).max()


def test_carriage_refuses_other_solvers_starts_and_split_stages():
    wl = carriage()
    for over in (dict(solver=oracle.SOLVER_NEWTON), dict(solver=oracle.SOLVER_GS), dict(warm=oracle.WARM_PREV)):
        with pytest.raises(ValueError):
            oracle.Oracle(wl, **over)
    o = oracle.Oracle(wl)
    for stage in (lambda: o.predict(0, 0.01), lambda: o.pre_substep(0, 0), lambda: o.solve_substep(0, o.q)):
        with pytest.raises(ValueError):
            stage()


def test_first_iteration_is_the_scaled_block_solve():
    """From zero multipliers one iteration gives every block
    dl = -(relax / d) K^-1 C, K = J_blk W J_blk^T + diag(alpha~), at the
    predicted state, d the largest block count of its bodies (counted here
    from the nonzero columns of the assembled J: a segment carries its
    joints and its wheels' hinge blocks, a wheel its hinge blocks and its
    contact); the hinge axis block uses its two rigid rows; a contact block
    takes the normal row by K_nn and the tangential pair by its 2x2 block,
    then the Coulomb disc of radius mu lambda_n."""
    wl = carriage(n_modules=(1,), segs=(3,), substeps=1, relax=0.8)
    o = oracle.Oracle(wl)
    o.cmd[...] = 0.5
    o.v[:, 0] = 0.01
    o.wv[:, 0] = 0.01
    o.run(3)
    st = {k: getattr(o, k).copy() for k in ("x", "q", "v", "w", "wx", "wq", "wv", "ww")}
    one = oracle.Oracle(wl, iters=1, tol=0.0)
    for k, v in st.items():
        getattr(one, k)[...] = v
    one.p[...] = o.p
    one.cmd[...] = o.cmd
    one.run(1)
    B = int(one.B[0])
    xs, qs = np.r_[st["x"], st["wx"]], np.r_[st["q"], st["wq"]]
    xt, qt, _, _ = one.predict_bodies(0, xs, qs, np.r_[st["v"], st["wv"]], np.r_[st["w"], st["ww"]], wl.dt)
    Cv, J, Wm, comp = one.assemble_wheels(0, xt, qt, xs, qs, one.p)
    nblk = len(Cv) // 3
    touches = [sorted({c // 6 for c in np.nonzero(np.abs(J[3 * n:3 * n + 3]).sum(axis=0))[0]}) for n in range(nblk)]
    deg = np.zeros(3 * B, int)
    for t in touches:
        deg[t] += 1
    assert list(deg[:B]) == [6, 8, 6] and np.all(deg[B:] == 3)
    nj = 2 * (B - 1)
    expect = np.zeros(3 * nblk)
    mu = float(wl.mu[0])
    for n in range(nblk):
        sc = 0.8 / max(deg[b] for b in touches[n])
        rows = np.arange(3 * n, 3 * n + 3)
        kind = None if n < nj else (n - nj) % 3
        if kind == 1:
            rows = rows[[0, 2]]
        if kind == 2:
            K = J[rows] @ Wm @ J[rows].T
            ln = max(0.0, -sc * Cv[rows[0]] / K[0, 0])
            lt = -sc * np.linalg.solve(K[1:, 1:], Cv[rows[1:]])
            if np.linalg.norm(lt) > mu * ln:
                lt *= mu * ln / np.linalg.norm(lt)
            expect[rows] = [ln, *lt]
            continue
        K = J[rows] @ Wm @ J[rows].T + np.diag(comp[rows])
        expect[rows] = -sc * np.linalg.solve(K, Cv[rows])
    got = np.r_[one.lam_j.reshape(-1), one.lam_w.reshape(-1)]
    assert np.abs(expect).max() > 0 and np.any(expect[3 * nj + 6::9] > 0)
    assert np.abs(got - expect).max() <= 1e-9 * np.abs(expect).max()
