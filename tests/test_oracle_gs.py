"""Pins of the oracle's block Gauss-Seidel solver (block solves of the
compliant system visited colour by colour over the greedy block colouring).

A dense direct solve of eq. schur_system, and agreement with the
independent block-Jacobi iteration on the linearised problem with contact
and Coulomb friction (one solution), pin it; the colour-by-colour order is
pinned by the sweep count it needs against Jacobi's."""
import numpy as np
import pytest

import oracle
import workloads as W


def gs(wl, **kw):
    return oracle.Oracle(wl, solver=oracle.SOLVER_GS, **kw)


def snapshot(o):
    return {k: getattr(o, k).copy() for k in ("x", "q", "v", "w", "p", "cmd", "lam_j", "lam_c", "step")}


def load(o, st):
    for k, v in st.items():
        getattr(o, k)[...] = v
    return o


def test_gs_reaches_the_dense_solve_without_contact():
    """Linearised, no ground: the sweeps converge to dl = A^-1 (-C) with
    A = J W J^T + alpha~ assembled densely at the predicted state."""
    wl = W.make("short", n_snakes=2)
    kw = dict(substeps=1, flags=wl.flags | oracle.FLAG_NO_GROUND | oracle.FLAG_LINEARISED,
              controller=W.CTRL_EXTERNAL)
    o = oracle.Oracle(wl, **kw)
    o.cmd[...] = 0.3
    o.run(3)
    st = snapshot(o)
    g = load(gs(wl, tol=0, iters=3000, **kw), st)
    g.run(1)
    for s in range(g.n):
        a, b = g.body_off[s], g.body_off[s + 1]
        pred = load(oracle.Oracle(wl, **kw), st).predict(s, wl.dt)
        Cv, J, Wm, comp = g.assemble(s, pred["x"].copy(), pred["q"].copy(), st["x"][a:b], g.snake(s)["p"])
        dl = np.linalg.solve(J @ Wm @ J.T + np.diag(comp), -Cv)
        lam = g.snake(s)["lam_j"].reshape(-1)
        assert np.abs(lam - dl).max() <= 1e-9 * np.abs(dl).max()
        assert g.residual[s] < 1e-13


def test_gs_meets_block_jacobi_on_the_linearised_problem():
    """With contact and friction the linearised problem has one solution:
    Gauss-Seidel and Jacobi, run to 1e-12, agree, Gauss-Seidel in under a
    fifth of the sweeps."""
    wl = W.make("short", n_snakes=8)
    kw = dict(substeps=1, flags=wl.flags | oracle.FLAG_LINEARISED)
    o = oracle.Oracle(wl, **kw)
    o.run(20)
    st = snapshot(o)
    j = load(oracle.Oracle(wl, tol=1e-12, iters=3_000_000, **kw), st)
    g = load(gs(wl, tol=1e-12, iters=3_000_000, **kw), st)
    for s in (3, 4):
        j.run(1, snakes=(s, s + 1))
        g.run(1, snakes=(s, s + 1))
        assert j.status[s] == 0 and g.status[s] == 0
        assert g.iters[s] * 5 < j.iters[s]
        dj, dg = j.snake(s), g.snake(s)
        assert np.abs(dg["x"] - dj["x"]).max() <= 1e-10
        for k in ("lam_j", "lam_c"):
            assert np.abs(dg[k] - dj[k]).max() <= 1e-7 * np.abs(dj[k]).max(), k


def test_gs_budget_counts_sweeps():
    wl = W.make("uneven", n_snakes=3)
    o = gs(wl, tol=0, iters=7)
    o.run(2)
    assert np.all(o.iters == 7 * wl.substeps)
    assert np.all(np.isfinite(o.x))


def greedy_colours(nj):
    """Greedy colouring of a chain's blocks in block order (stretch_j,
    bend_j per joint j, bodies j and j+1): smallest colour unused by an
    earlier block sharing a body."""
    bodies = [(j, j + 1) for j in range(nj) for _ in range(2)]
    col = []
    for k, bk in enumerate(bodies):
        taken = {col[e] for e in range(k) if set(bodies[e]) & set(bk)}
        c = 0
        while c in taken:
            c += 1
        col.append(c)
    return np.array(col)


@pytest.mark.parametrize("relax", [1.0, 0.7])
def test_gs_sweeps_are_block_gauss_seidel_in_colour_order(relax):
    """Linearised, no ground: a sweep is the block successive
    over-relaxation of the dense system A l = -C (3x3 diagonal blocks solved
    exactly, l_i <- (1 - w) l_i + w A_ii^-1 (-C_i - sum_j!=i A_ij l_j),
    w = relax; Gauss-Seidel at w = 1), blocks taken in colour order (by
    block index within a colour); checked after one, two and three sweeps."""
    wl = W.make("short", n_snakes=2)
    kw = dict(substeps=1, flags=wl.flags | oracle.FLAG_NO_GROUND | oracle.FLAG_LINEARISED,
              controller=W.CTRL_EXTERNAL, relax=relax)
    o = oracle.Oracle(wl, **kw)
    o.cmd[...] = 0.3
    o.run(3)
    st = snapshot(o)
    for s in range(o.n):
        a, b = o.body_off[s], o.body_off[s + 1]
        pred = load(oracle.Oracle(wl, **kw), st).predict(s, wl.dt)
        stepped = load(gs(wl, tol=0, iters=1, **kw), st)
        stepped.run(1)   # pressures of the substep (the lag moves them first)
        Cv, J, Wm, comp = o.assemble(s, pred["x"].copy(), pred["q"].copy(), st["x"][a:b],
                                     stepped.snake(s)["p"])
        A = J @ Wm @ J.T + np.diag(comp)
        nblk = len(Cv) // 3
        order = np.argsort(greedy_colours(nblk // 2), kind="stable")
        lam = np.zeros(len(Cv))
        for sweeps in (1, 2, 3):
            for k in order:
                r = slice(3 * k, 3 * k + 3)
                rest = A[r] @ lam - A[r, r] @ lam[r]
                lam[r] = (1 - relax) * lam[r] + relax * np.linalg.solve(A[r, r], -Cv[r] - rest)
            g = load(gs(wl, tol=0, iters=sweeps, **kw), st)
            g.run(1)
            got = g.snake(s)["lam_j"].reshape(-1)
            assert np.abs(got - lam).max() <= 1e-9 * np.abs(lam).max(), sweeps
