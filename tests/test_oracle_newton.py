"""Pins of the oracle's Newton solver (section "Time-Stepping": Newton
iterations, each solving eq. schur_system with preconditioned conjugate-residual
iterations; contact through a Fischer-Burmeister reformulation).

None of them re-types the solver: a dense direct solve of eq. schur_system,
the quadratic convergence of Newton's method on the smooth (contact-free)
problem, and agreement with the independent block-Jacobi iteration on the
linearised problem, whose solution (with contact and Coulomb friction) is
unique, pin it.
"""
import numpy as np

import oracle
import workloads as W


def newton(wl, **kw):
    return oracle.Oracle(wl, solver=oracle.SOLVER_NEWTON, **kw)


def moved_state(wl, **kw):
    """State after a few plain steps (off the initial straight chain)."""
    o = oracle.Oracle(wl, **kw)
    o.run(6)
    return {k: getattr(o, k).copy() for k in ("x", "q", "v", "w", "p", "cmd", "lam_j", "lam_c", "step")}


def load(o, st):
    for k, v in st.items():
        getattr(o, k)[...] = v
    return o


def test_one_newton_step_is_the_dense_solve_of_the_schur_system():
    """Without contact, one Newton iteration from zero multipliers with an
    inner solve run to convergence gives dl = A^-1 (-C) with
    A = J W J^T + alpha~ assembled densely at the predicted state, and
    x = x~ + (W J^T dl)_x."""
    wl = W.make("short", n_snakes=2)
    kw = dict(substeps=1, flags=wl.flags | oracle.FLAG_NO_GROUND, controller=W.CTRL_EXTERNAL)
    st = moved_state(wl, **kw)
    o = load(newton(wl, newton_iters=1, pcr_iters=400, tol=0, **kw), st)
    o.run(1)
    for s in range(o.n):
        a, b = o.body_off[s], o.body_off[s + 1]
        pr = load(oracle.Oracle(wl, **kw), st)
        pred = pr.predict(s, wl.dt)
        xt, qt = pred["x"].copy(), pred["q"].copy()
        Cv, J, Wm, comp = o.assemble(s, xt, qt, st["x"][a:b], o.snake(s)["p"])
        dl = np.linalg.solve(J @ Wm @ J.T + np.diag(comp), -Cv)
        dx = (Wm @ J.T @ dl).reshape(b - a, 6)[:, :3]
        lam = o.snake(s)["lam_j"].reshape(-1)
        assert np.abs(lam - dl).max() <= 1e-10 * np.abs(dl).max()
        assert np.abs(o.snake(s)["x"] - (xt + dx)).max() <= 1e-12
        assert o.iters[s] == 400


def test_newton_converges_quadratically_without_contact():
    """On the smooth problem (no ground) Newton's method with exact inner
    solves reaches round-off within three iterations from a residual of
    order 1e-3."""
    wl = W.make("short", n_snakes=4)
    kw = dict(flags=wl.flags | oracle.FLAG_NO_GROUND)
    st = moved_state(wl, **kw)
    r = []
    for k in (0, 1, 3):
        o = load(newton(wl, newton_iters=k, pcr_iters=300, tol=0, substeps=1, **kw), st)
        o.run(1)
        r.append(o.residual.copy())
    assert np.all(r[0] > 1e-5)
    assert np.all(r[1] < r[0])
    assert np.all(r[2] < 1e-12)


def test_newton_meets_block_jacobi_on_the_linearised_problem():
    """With the Jacobians frozen at the predicted state the problem (joints,
    unilateral contact, Coulomb friction) has one solution; Newton's method
    with the Fischer-Burmeister and natural-map rows and block-Jacobi
    iterations, two different algorithms, must both reach it.  (Without a
    line search the Newton iterates of some substeps cycle between stick and
    slip instead; the two snakes checked here are ones where they do not.)"""
    wl = W.make("short", n_snakes=8)
    kw = dict(substeps=1, flags=wl.flags | oracle.FLAG_LINEARISED)
    o = oracle.Oracle(wl, **kw)
    o.run(20)
    st = {k: getattr(o, k).copy() for k in ("x", "q", "v", "w", "p", "cmd", "lam_j", "lam_c", "step")}
    pick = [3, 7]
    j = load(oracle.Oracle(wl, tol=1e-12, iters=3_000_000, **kw), st)
    n = load(newton(wl, newton_iters=60, pcr_iters=300, tol=0, **kw), st)
    for s in pick:
        j.run(1, snakes=(s, s + 1))
        n.run(1, snakes=(s, s + 1))
        assert j.step[s] == st["step"][s] + 1 and n.step[s] == st["step"][s] + 1
        assert j.status[s] == 0
        assert n.residual[s] < 1e-12
        dn, dj = n.snake(s), j.snake(s)
        assert np.abs(dn["x"] - dj["x"]).max() <= 1e-9
        for k in ("lam_j", "lam_c"):
            assert np.abs(dn[k] - dj[k]).max() <= 1e-6 * np.abs(dj[k]).max(), k


def test_newton_with_frictionless_contact_converges():
    """Frictionless ground contact alone (the Fischer-Burmeister rows) keeps
    Newton's method convergent: residual below 1e-9 after 12 iterations."""
    wl = W.make("short", n_snakes=4)
    wl.mu = np.zeros(len(wl.n_modules))
    st = moved_state(wl)
    o = load(newton(wl, newton_iters=12, pcr_iters=300, tol=0), st)
    o.run(1)
    assert np.all(o.residual < 1e-9)


def test_newton_budget_and_tolerance():
    """A fixed budget reports newton_iters * pcr_iters inner iterations per
    substep; with a tolerance the solve stops at the first Newton iterate
    whose residual is below it, counting only the inner iterations run."""
    wl = W.make("short", n_snakes=3)
    st = moved_state(wl)
    o = load(newton(wl, newton_iters=4, pcr_iters=20, tol=0), st)
    o.run(1)
    assert np.all(o.iters == 4 * 20 * wl.substeps)
    o = load(newton(wl, newton_iters=40, pcr_iters=100, tol=1e-6,
                    flags=wl.flags | oracle.FLAG_NO_GROUND), st)
    o.run(1)
    assert np.all(o.residual <= 1e-6) and np.all(o.status == 0)
    assert np.all(o.iters % 100 == 0) and np.all(o.iters < 40 * 100 * wl.substeps)


def test_newton_previous_multipliers_start_as_jacobi_does():
    """The previous-multiplier start moves the predicted bodies by
    W J(x~)^T lambda0, as the Jacobi solver's does (pinned with it): zero
    Newton iterations from it give the Jacobi solver's zero-iteration state
    and residual exactly, and from zero multipliers it is the zero start
    (up to the renormalisation of a zero turn)."""
    wl = W.make("short", n_snakes=4)
    st = moved_state(wl)
    assert np.abs(st["lam_j"]).max() > 0 and np.abs(st["lam_c"]).max() > 0
    p = load(newton(wl, newton_iters=0, pcr_iters=1, tol=0, warm=oracle.WARM_PREV), st)
    p.run(1)
    j = load(oracle.Oracle(wl, iters=0, tol=0, warm=oracle.WARM_PREV), st)
    j.run(1)
    for k in ("x", "q", "lam_j", "lam_c", "residual"):
        assert np.array_equal(getattr(p, k), getattr(j, k)), k
    zero = dict(st, lam_j=np.zeros_like(st["lam_j"]), lam_c=np.zeros_like(st["lam_c"]))
    a = load(newton(wl, warm=oracle.WARM_PREV, substeps=1), zero)
    a.run(1)
    b = load(newton(wl, substeps=1), zero)
    b.run(1)
    # (equal up to the renormalisation of q after a zero turn)
    assert np.array_equal(a.iters, b.iters)
    for k in ("x", "q", "lam_j", "lam_c"):
        ref = np.abs(getattr(b, k)).max()
        assert np.abs(getattr(a, k) - getattr(b, k)).max() <= 1e-9 * ref, k


def test_newton_keep_best_ends_at_the_best_iterate():
    """With newton_keep_best the substep ends at the Newton iterate of
    smallest residual: the same state, bit for bit, as the plain solve
    stopped after that many iterations (found by separate runs with 0..N
    iterations); the inner iterations of all N still count."""
    wl = W.make("short", n_snakes=8)
    kw = dict(substeps=1, tol=0, pcr_iters=20)
    st = moved_state(wl, substeps=1)
    N = 8
    runs = []
    for k in range(N + 1):
        o = load(newton(wl, newton_iters=k, **kw), st)
        o.run(1)
        runs.append(o)
    kb = load(newton(wl, newton_iters=N, newton_keep_best=1, **kw), st)
    kb.run(1)
    assert np.all(kb.iters == N * 20)
    cycled = 0
    for s in range(wl.n_snakes):
        r = np.array([o.residual[s] for o in runs])
        best = int(np.argmin(r))          # the earliest of equal minima
        cycled += best < N
        assert kb.residual[s] == r[best]
        d, ref = kb.snake(s), runs[best].snake(s)
        for f in ("x", "q", "lam_j", "lam_c"):
            assert np.array_equal(d[f], ref[f]), (s, f)
    assert cycled > 0   # some snake's last iterate is not its best


def test_friction_trial_scale_sweep():
    """Reading of the friction natural map's trial scale m' (the paper names
    no reformulation for the cone).  Every positive m' has the same roots,
    but the scale decides how the semismooth iterates behave, and the two
    ends pull apart.  Measured (largest-residual medians / maxima after
    4 x 20 Newton x PCR iterations on 64 snakes six steps in; full solves:
    snakes of the linearised problem below reaching 1e-12 in 60 Newton
    iterations):

        m'      short        uniform      uneven       full solves
        1       0.37 / 6.1   0.13 / 0.61  0.20 / 0.66  7 / 8
        3       0.019 / 1.1  0.056 / 0.32 0.085 / 0.21 6 / 8
        10      0.011 / 1.5  0.055 / 0.42 0.061 / 0.16 6 / 8
        30      0.0065/ 0.12 0.055 / 0.16 0.055 / 0.16 3 / 8
        100     0.0061/ 0.085 0.055/ 0.17 0.055 / 0.12 1 / 8
        1000    0.0070/ 0.045 0.055/ 0.30 0.056 / 0.12 0 / 8

    One body mass leaves the short snakes' contacts cycling at the paper's
    budget; from thirty masses up the full solves cycle instead.  Ten masses
    (the oracle's and the kernel's value) is the compromise; the test holds
    the three corners of that trade."""
    from parity import load_oracle, rounded_state

    L = oracle.lib()
    assert L.orc_set_friction_trial(10.0) == 10.0      # the default
    try:
        wl8 = W.make("short", n_snakes=8)
        kw = dict(substeps=1, flags=wl8.flags | oracle.FLAG_LINEARISED)
        lin = oracle.Oracle(wl8, **kw)
        lin.run(20)
        st8 = {k: getattr(lin, k).copy() for k in ("x", "q", "v", "w", "p", "cmd", "lam_j", "lam_c", "step")}
        wl = W.make("short", n_snakes=64)
        base = oracle.Oracle(wl)
        base.run(6, threads=8)
        base.commands()
        st = rounded_state(base)
        full, budget = {}, {}
        for scale in (1.0, 10.0, 100.0):
            L.orc_set_friction_trial(scale)
            n = load(newton(wl8, newton_iters=60, pcr_iters=300, tol=0, **kw), st8)
            n.run(1)
            full[scale] = int((n.residual < 1e-12).sum())
            o = oracle.Oracle(wl, solver=oracle.SOLVER_NEWTON, newton_iters=4, pcr_iters=20, tol=0.0,
                              controller=W.CTRL_EXTERNAL)
            load_oracle(o, st)
            o.step[:] = base.step
            o.run(1, threads=8)
            budget[scale] = (float(np.median(o.residual)), float(o.residual.max()))
        print("\n[friction trial] full solves", full, "budget median/max", budget)
        assert budget[1.0][0] > 0.1 and budget[1.0][1] > 1.0        # cycles at the budget
        assert full[10.0] >= 6 and budget[10.0][0] < 0.05            # the compromise
        assert full[100.0] <= 2                                      # full solves cycle
    finally:
        L.orc_set_friction_trial(10.0)
