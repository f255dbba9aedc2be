"""Python handle on the FP64 CPU oracle (``snake_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline
leg of the benchmark use it; the GPU library never imports, links or runs
anything in this folder, and this folder imports nothing from the GPU
library.  Inputs come from the shared seeded generator in ``workloads``.

State arrays here are array-of-structures per body, float64:
``x[N,3]``, ``q[N,4]`` (w,x,y,z), ``v[N,3]``, ``w[N,3]``, ``p[Mtot,2]``,
``cmd[Mtot]``, ``lam_j[Jtot,6]`` (stretch xyz, twist, bend_y, bend_z) and
``lam_c[N,3]`` (normal, tangential x, tangential y).  A wheel carriage
(``FLAG_WHEELS``) adds ``wx[2N,3]``, ``wq[2N,4]``, ``wv``, ``ww`` (wheel 2i+k
of body i) and ``lam_w[2N,9]`` (hinge position, hinge axis, contact).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "snake_oracle.c")
SRCS = [SRC, os.path.join(HERE, "mlp_oracle.c"), os.path.join(HERE, "fem_oracle.c"),
        os.path.join(HERE, "link_oracle.c")]
# SNAKE_SANITIZE=1 selects the sanitizer build (AddressSanitizer and
# UndefinedBehaviorSanitizer with the shared runtime, which the process must
# preload), made by tests/run_sanitizers.py.  CPU only.
SANITIZE = os.environ.get("SNAKE_SANITIZE") == "1"
LIB = os.path.join(HERE, "liboracle_san.so" if SANITIZE else "liboracle.so")

FLAG_FIXED_ROOT = 1
FLAG_NO_GROUND = 2
FLAG_LINEARISED = 8
FLAG_WHEELS = 16
WARM_ZERO, WARM_PREV, WARM_GIVEN = 0, 1, 2
STATUS_NONFINITE, STATUS_NOT_CONVERGED = 1, 2
SOLVER_JACOBI, SOLVER_NEWTON, SOLVER_GS = 0, 1, 2

_lock = threading.Lock()
_lib = None


def build(force: bool = True, cc=("gcc",)) -> str:
    """Compile the oracle (gcc -O2, no fast-math; ``cc`` replaces the
    compiler and adds flags, as the sanitizer build does)."""
    if force or _stale():
        if SANITIZE and tuple(cc) == ("gcc",):
            raise RuntimeError("the sanitizer build of the oracle is made by tests/run_sanitizers.py")
        tmp = LIB + ".tmp"
        subprocess.check_call([*cc, "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, *SRCS, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _stale():
    return not os.path.exists(LIB) or any(os.path.getmtime(LIB) < os.path.getmtime(s) for s in SRCS)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if _stale():
                build(force=True)
            _lib = C.CDLL(LIB)
            _declare(_lib)
    return _lib


_P = C.c_void_p


class Batch(C.Structure):
    _fields_ = [
        ("n_snakes", C.c_int32),
        ("n_modules", _P), ("segs", _P),
        ("alpha_s", _P), ("alpha_b", _P), ("alpha_t", _P), ("mu", _P),
        ("freq", _P), ("phase0", _P),
        ("sched_off", _P), ("sched_steps", _P), ("sched_val", _P),
        ("mass", C.c_double), ("length", C.c_double), ("radius", C.c_double),
        ("gravity", C.c_double),
        ("dt", C.c_double),
        ("substeps", C.c_int32), ("iters", C.c_int32),
        ("tol", C.c_double), ("relax", C.c_double),
        ("law", C.c_int32),
        ("tau_inf", C.c_double), ("tau_def", C.c_double), ("kappa_max", C.c_double),
        ("k_i", C.c_double), ("k_d", C.c_double), ("T_p", C.c_double), ("p_s", C.c_double),
        ("amp_psi", C.c_double),
        ("flags", C.c_int32), ("controller", C.c_int32), ("warm", C.c_int32),
        ("ctrl_alpha", C.c_double), ("ctrl_offset", C.c_double),
        ("fallback", C.c_int32), ("fallback_k", C.c_int32),
        ("solver", C.c_int32), ("newton_iters", C.c_int32), ("pcr_iters", C.c_int32),
        ("newton_keep_best", C.c_int32),
    ]


class State(C.Structure):
    _fields_ = [(n, _P) for n in ("x", "q", "v", "w", "p", "cmd", "lam_j", "lam_c",
                                  "residual", "iters", "status", "iters_total", "step",
                                  "wx", "wq", "wv", "ww", "lam_w")]


def _declare(L):
    bp, sp = C.POINTER(Batch), C.POINTER(State)
    L.orc_offsets.argtypes = [bp, _P, _P, _P, _P]
    L.orc_set_friction_trial.argtypes = [C.c_double]
    L.orc_set_friction_trial.restype = C.c_double
    L.orc_init_state.argtypes = [bp, sp]
    L.orc_commands.argtypes = [bp, sp, C.c_int32, C.c_int32]
    L.orc_run.argtypes = [bp, sp, C.c_int32, C.c_int32, C.c_int32]
    L.orc_run.restype = C.c_int
    L.orc_assemble.argtypes = [bp, C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P]
    L.orc_assemble.restype = C.c_int
    L.orc_assemble_wheels.argtypes = [bp, C.c_int32] + [_P] * 9
    L.orc_assemble_wheels.restype = C.c_int
    L.orc_predict_snake.argtypes = [bp, C.c_int32, _P, _P, _P, _P, C.c_double]
    L.orc_index.argtypes = [bp] + [_P] * 7
    L.orc_pre_substep.argtypes = [bp, C.c_int32, C.c_int32] + [_P] * 7
    L.orc_solve_substep.argtypes = [bp, C.c_int32] + [_P] * 11
    L.orc_features.argtypes = [bp, C.c_int32] + [_P] * 9
    L.orc_targets.argtypes = [bp, C.c_int32, _P, _P, _P]
    L.fem_tet_rest.argtypes = [_P, _P, _P]
    L.fem_tet_rest.restype = C.c_int
    L.fem_polar.argtypes = [_P, _P]
    L.fem_polar.restype = C.c_int
    L.fem_tet_eval.argtypes = [_P, _P, _P, C.c_int, _P, _P]
    L.fem_tet_eval.restype = C.c_int
    L.fem_tet_compliance.argtypes = [C.c_double, C.c_double, C.c_double, _P]
    L.fem_expansion.argtypes = [C.c_double, C.c_double]
    L.fem_expansion.restype = C.c_double
    L.fem_dist_eval.argtypes = [_P, _P, C.c_double, C.c_double, C.c_double, _P]
    L.fem_dist_eval.restype = C.c_double
    L.fem_attach_eval.argtypes = [_P] * 6
    L.mlo_param_count.restype = C.c_int
    L.mlo_norm_stats.argtypes = [_P, C.c_int64, _P, _P]
    L.mlo_forward.argtypes = [_P, _P, _P, _P, C.c_int64, _P]
    L.mlo_loss_grad.argtypes = [_P, _P, _P, _P, _P, C.c_int64, _P]
    L.mlo_loss_grad.restype = C.c_double
    L.mlo_grad_abs.argtypes = [_P, _P, _P, _P, _P, C.c_int64, _P]
    L.mlo_adam.argtypes = [_P, _P, _P, _P, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                           C.c_double]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Oracle:
    """An FP64 batch built from a ``workloads.Workload`` (or any object with
    the same fields).  Keyword overrides replace workload settings."""

    def __init__(self, wl, **over):
        self.L = lib()
        g = lambda k: over.get(k, getattr(wl, k))  # noqa: E731
        self._keep = {}

        def arr(name, a, dt):
            a = np.ascontiguousarray(np.asarray(a, dtype=dt))
            self._keep[name] = a
            return _ptr(a)

        n = int(len(wl.n_modules))
        b = Batch()
        b.n_snakes = n
        b.n_modules = arr("nm", g("n_modules"), np.int32)
        b.segs = arr("sg", g("segs_per_module"), np.int32)
        b.alpha_s = arr("as", g("alpha_stretch"), np.float64)
        b.alpha_b = arr("ab", g("alpha_bend"), np.float64)
        b.alpha_t = arr("at", g("alpha_twist"), np.float64)
        b.mu = arr("mu", g("mu"), np.float64)
        b.freq = arr("fr", g("ctrl_freq"), np.float64)
        b.phase0 = arr("ph", g("ctrl_phase0"), np.float64)
        so = g("sched_off")
        if so is not None:
            b.sched_off = arr("so", so, np.int32)
            b.sched_steps = arr("ss", g("sched_steps"), np.int32)
            b.sched_val = arr("sv", g("sched_val"), np.float64)
        for f, k in (("mass", "seg_mass"), ("length", "seg_length"), ("radius", "seg_radius"),
                     ("gravity", "gravity"), ("dt", "dt"), ("tol", "tol"), ("relax", "relax"),
                     ("tau_inf", "tau_inflate"), ("tau_def", "tau_deflate"),
                     ("kappa_max", "kappa_max"), ("k_i", "k_inflate"), ("k_d", "k_deflate"),
                     ("T_p", "T_p"), ("p_s", "p_source"), ("amp_psi", "amplitude_psi"),
                     ("ctrl_alpha", "ctrl_alpha"), ("ctrl_offset", "ctrl_offset")):
            setattr(b, f, float(g(k)))
        b.substeps = int(g("substeps"))
        b.iters = int(g("iters"))
        b.law = int(g("pressure_law"))
        b.flags = int(g("flags"))
        b.controller = int(g("controller"))
        b.warm = int(over.get("warm", WARM_ZERO))
        b.fallback = int(over.get("fallback", 0))
        b.fallback_k = int(over.get("fallback_k", 0))
        b.solver = int(over.get("solver", getattr(wl, "solver", SOLVER_JACOBI)))
        b.newton_iters = int(over.get("newton_iters", getattr(wl, "newton_iters", 4)))
        b.pcr_iters = int(over.get("pcr_iters", getattr(wl, "pcr_iters", 20)))
        b.newton_keep_best = int(over.get("newton_keep_best", 0))
        self.batch = b
        self.n = n
        self.B = (np.asarray(g("n_modules"), np.int64) * np.asarray(g("segs_per_module"), np.int64))
        self.M = np.asarray(g("n_modules"), np.int64)
        self.body_off = np.zeros(n + 1, np.int64)
        self.joint_off = np.zeros(n + 1, np.int64)
        self.module_off = np.zeros(n + 1, np.int64)
        self.block_off = np.zeros(n + 1, np.int64)
        self.L.orc_offsets(C.byref(b), _ptr(self.body_off), _ptr(self.joint_off),
                           _ptr(self.module_off), _ptr(self.block_off))
        N, J, Mt = int(self.body_off[-1]), int(self.joint_off[-1]), int(self.module_off[-1])
        self.x = np.zeros((N, 3))
        self.q = np.zeros((N, 4))
        self.v = np.zeros((N, 3))
        self.w = np.zeros((N, 3))
        self.p = np.zeros((Mt, 2))
        self.cmd = np.zeros(Mt)
        self.lam_j = np.zeros((max(J, 0), 6))
        self.lam_c = np.zeros((N, 3))
        self.residual = np.zeros(n)
        self.iters = np.zeros(n, np.int32)
        self.status = np.zeros(n, np.int32)
        self.iters_total = np.zeros(n, np.int64)
        self.step = np.zeros(n, np.int64)
        self.wheels = bool(b.flags & FLAG_WHEELS)
        if self.wheels:
            if b.solver != SOLVER_JACOBI or b.warm != WARM_ZERO:
                raise ValueError("a wheel carriage takes the Jacobi solver from the zero start")
            self.wx = np.zeros((2 * N, 3))
            self.wq = np.zeros((2 * N, 4))
            self.wv = np.zeros((2 * N, 3))
            self.ww = np.zeros((2 * N, 3))
            self.lam_w = np.zeros((2 * N, 9))
        self._state()
        self.L.orc_init_state(C.byref(self.batch), C.byref(self.st))

    def _state(self):
        s = State()
        for f in ("x", "q", "v", "w", "p", "cmd", "lam_j", "lam_c", "residual", "iters",
                  "status", "iters_total", "step"):
            setattr(s, f, _ptr(getattr(self, f)))
        if self.wheels:
            for f in ("wx", "wq", "wv", "ww", "lam_w"):
                setattr(s, f, _ptr(getattr(self, f)))
        self.st = s

    # -- stepping ---------------------------------------------------------
    def commands(self):
        self.L.orc_commands(C.byref(self.batch), C.byref(self.st), 0, self.n)
        return self.cmd

    def run(self, n_steps: int, threads: int = 1, snakes=None):
        """Advance snakes (default all) by ``n_steps`` steps.  With threads > 1
        contiguous snake ranges run concurrently (ctypes releases the GIL)."""
        s0, s1 = (0, self.n) if snakes is None else snakes
        if threads <= 1 or s1 - s0 <= 1:
            if self.L.orc_run(C.byref(self.batch), C.byref(self.st), s0, s1, int(n_steps)) != 0:
                raise ValueError("orc_run refused the batch")
            return self
        cost = self.B[s0:s1].astype(np.float64)
        cuts = np.searchsorted(np.cumsum(cost), np.linspace(0, cost.sum(), threads + 1)[1:-1])
        bounds = [s0] + [s0 + int(c) + 1 for c in cuts] + [s1]
        bounds = sorted(set(min(max(b, s0), s1) for b in bounds))
        with ThreadPoolExecutor(max_workers=threads) as ex:
            futs = [ex.submit(self.L.orc_run, C.byref(self.batch), C.byref(self.st), a, b, int(n_steps))
                    for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
            for f in futs:
                f.result()
        return self

    # -- per-snake views ----------------------------------------------------
    def snake(self, s: int) -> dict:
        b0, b1 = self.body_off[s], self.body_off[s + 1]
        j0, j1 = self.joint_off[s], self.joint_off[s + 1]
        m0, m1 = self.module_off[s], self.module_off[s + 1]
        d = dict(x=self.x[b0:b1], q=self.q[b0:b1], v=self.v[b0:b1], w=self.w[b0:b1],
                 p=self.p[m0:m1], cmd=self.cmd[m0:m1], lam_j=self.lam_j[j0:j1],
                 lam_c=self.lam_c[b0:b1])
        if self.wheels:
            d.update(wx=self.wx[2 * b0:2 * b1], wq=self.wq[2 * b0:2 * b1], wv=self.wv[2 * b0:2 * b1],
                     ww=self.ww[2 * b0:2 * b1], lam_w=self.lam_w[2 * b0:2 * b1])
        return d

    def assemble(self, s, x, q, xp, p):
        """Dense C, J, W, comp of snake s at configuration (x, q)."""
        B = int(self.B[s])
        ground = 0 if (self.batch.flags & FLAG_NO_GROUND) else 1
        rows = 6 * (B - 1) + (3 * B if ground else 0)
        Cv = np.zeros(rows)
        J = np.zeros((rows, 6 * B))
        W = np.zeros((6 * B, 6 * B))
        comp = np.zeros(rows)
        x, q, xp, p = (np.ascontiguousarray(a, np.float64) for a in (x, q, xp, p))
        self.L.orc_assemble(C.byref(self.batch), int(s), _ptr(x), _ptr(q), _ptr(xp), _ptr(p),
                            _ptr(Cv), _ptr(J), _ptr(W), _ptr(comp))
        return Cv, J, W, comp

    def assemble_wheels(self, s, x, q, xp, qp, p):
        """Dense C, J, W, comp of wheel-carriage snake s: x, q, xp, qp hold
        its B segments then its 2B wheels; 3 rows per block (a hinge axis
        block's spin row is all zero)."""
        B = int(self.B[s])
        ground = 0 if (self.batch.flags & FLAG_NO_GROUND) else 1
        rows = 6 * (B - 1) + 3 * 2 * B * (2 + ground)
        ncol = 6 * 3 * B
        Cv, J, W, comp = np.zeros(rows), np.zeros((rows, ncol)), np.zeros((ncol, ncol)), np.zeros(rows)
        x, q, xp, qp, p = (np.ascontiguousarray(a, np.float64) for a in (x, q, xp, qp, p))
        got = self.L.orc_assemble_wheels(C.byref(self.batch), int(s), _ptr(x), _ptr(q), _ptr(xp), _ptr(qp),
                                         _ptr(p), _ptr(Cv), _ptr(J), _ptr(W), _ptr(comp))
        assert got == rows
        return Cv, J, W, comp

    def predict_bodies(self, s, x, q, v, w, h):
        """The prediction stage on arrays holding all bodies of snake s (for
        a wheel carriage: segments, then wheels); returns new arrays."""
        arrs = [np.array(a, np.float64, order="C") for a in (x, q, v, w)]
        self.L.orc_predict_snake(C.byref(self.batch), int(s), *[_ptr(a) for a in arrs], float(h))
        return arrs

    def _plain_chain_only(self):
        if self.wheels:
            raise ValueError("this stage takes the plain chain; for a wheel carriage use predict_bodies / run")

    def predict(self, s, h):
        """Apply the prediction stage to snake s in place (returns its views)."""
        self._plain_chain_only()
        d = self.snake(s)
        arrs = [np.ascontiguousarray(d[k]) for k in ("x", "q", "v", "w")]
        self.L.orc_predict_snake(C.byref(self.batch), int(s), *[_ptr(a) for a in arrs], float(h))
        for k, a in zip(("x", "q", "v", "w"), arrs):
            d[k][...] = a
        return d

    # -- split substep (learned warm start) ------------------------------------
    def pre_substep(self, s, sub):
        """First half of substep `sub` of snake s in place; returns q_pred."""
        self._plain_chain_only()
        d = self.snake(s)
        arrs = {k: np.ascontiguousarray(d[k]) for k in ("x", "q", "v", "w", "p", "cmd")}
        qp = np.zeros_like(arrs["q"])
        self.L.orc_pre_substep(C.byref(self.batch), int(s), int(sub), *[_ptr(arrs[k]) for k in
                               ("x", "q", "v", "w", "p", "cmd")], _ptr(qp))
        for k in ("v", "w", "p"):
            d[k][...] = arrs[k]
        return qp

    def solve_substep(self, s, q_pred):
        """Second half for snake s (lam_* hold lambda0 for a GIVEN warm
        start); returns (residual, iterations, status)."""
        self._plain_chain_only()
        d = self.snake(s)
        arrs = {k: np.ascontiguousarray(d[k]) for k in ("x", "q", "v", "w", "p", "lam_j", "lam_c")}
        qp = np.ascontiguousarray(q_pred, np.float64)
        r, it, st = C.c_double(), C.c_int32(), C.c_int32()
        self.L.orc_solve_substep(C.byref(self.batch), int(s), _ptr(arrs["x"]), _ptr(arrs["q"]), _ptr(qp),
                                 _ptr(arrs["v"]), _ptr(arrs["w"]), _ptr(arrs["p"]), _ptr(arrs["lam_j"]),
                                 _ptr(arrs["lam_c"]), C.byref(r), C.byref(it), C.byref(st))
        for k in arrs:
            d[k][...] = arrs[k]
        return r.value, it.value, st.value

    def features(self, s, q_pred):
        d = self.snake(s)
        arrs = {k: np.ascontiguousarray(d[k]) for k in ("x", "v", "w", "p", "cmd", "lam_j", "lam_c")}
        B = int(self.B[s])
        out = np.zeros((2 * max(B - 1, 0), 32))
        qp = np.ascontiguousarray(q_pred, np.float64)
        self.L.orc_features(C.byref(self.batch), int(s), _ptr(arrs["x"]), _ptr(arrs["v"]), _ptr(arrs["w"]),
                            _ptr(qp), _ptr(arrs["p"]), _ptr(arrs["cmd"]), _ptr(arrs["lam_j"]),
                            _ptr(arrs["lam_c"]), _ptr(out))
        return out

    def targets(self, s, q_pred):
        d = self.snake(s)
        B = int(self.B[s])
        out = np.zeros((2 * max(B - 1, 0), 3))
        lj = np.ascontiguousarray(d["lam_j"])
        self.L.orc_targets(C.byref(self.batch), int(s), _ptr(np.ascontiguousarray(q_pred, np.float64)),
                           _ptr(lj), _ptr(out))
        return out

    def index(self):
        """Offsets, block list, degrees, greedy colours, buckets, work order."""
        nb = int(self.block_off[-1])
        N = int(self.body_off[-1])
        out = dict(blk_type=np.zeros(nb, np.int32), blk_a=np.zeros(nb, np.int32),
                   blk_b=np.zeros(nb, np.int32), blk_color=np.zeros(nb, np.int32),
                   body_degree=np.zeros(N, np.int32), bucket=np.zeros(self.n, np.int32),
                   order=np.zeros(self.n, np.int32))
        self.L.orc_index(C.byref(self.batch), *[_ptr(out[k]) for k in (
            "blk_type", "blk_a", "blk_b", "blk_color", "body_degree", "bucket", "order")])
        out.update(body_off=self.body_off.copy(), joint_off=self.joint_off.copy(),
                   module_off=self.module_off.copy(), block_off=self.block_off.copy())
        return out


# ---------------------------------------------------------------- MLP oracle

def _d(a):
    return np.ascontiguousarray(np.asarray(a, np.float64))


def mlp_param_count() -> int:
    return int(lib().mlo_param_count())


def mlp_norm_stats(x):
    x = _d(x)
    mean, std = np.zeros(32), np.zeros(32)
    lib().mlo_norm_stats(_ptr(x), x.shape[0], _ptr(mean), _ptr(std))
    return mean, std


def mlp_forward(params, mean, std, x):
    params, mean, std, x = _d(params), _d(mean), _d(std), _d(x)
    y = np.zeros((x.shape[0], 3))
    lib().mlo_forward(_ptr(params), _ptr(mean), _ptr(std), _ptr(x), x.shape[0], _ptr(y))
    return y


def mlp_loss_grad(params, mean, std, x, t, with_grad=True):
    params, mean, std, x, t = _d(params), _d(mean), _d(std), _d(x), _d(t)
    g = np.zeros(params.size) if with_grad else None
    loss = lib().mlo_loss_grad(_ptr(params), _ptr(mean), _ptr(std), _ptr(x), _ptr(t), x.shape[0],
                               _ptr(g))
    return loss, g


def mlp_grad_abs(params, mean, std, x, t):
    """Per-entry scale of the gradient's rounding error: the sum over samples
    of |delta| |activation|, deltas carried back through absolute values."""
    params, mean, std, x, t = _d(params), _d(mean), _d(std), _d(x), _d(t)
    A = np.zeros(params.size)
    lib().mlo_grad_abs(_ptr(params), _ptr(mean), _ptr(std), _ptr(x), _ptr(t), x.shape[0], _ptr(A))
    return A


def mlp_adam(params, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays."""
    lib().mlo_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(_d(g)), params.size, int(t), lr, b1, b2, eps)


# ---------------------------------------------------------------- link elements

def fem_tet_rest(X):
    """Rest tetrahedron X[4][3] -> (Dm^-1 [3][3], volume)."""
    X = _d(X)
    Dm_inv, V = np.zeros((3, 3)), C.c_double()
    if lib().fem_tet_rest(_ptr(X), _ptr(Dm_inv), C.byref(V)) != 0:
        raise ValueError("degenerate tetrahedron")
    return Dm_inv, V.value


def fem_polar(F):
    F, R = _d(F), np.zeros((3, 3))
    if lib().fem_polar(_ptr(F), _ptr(R)) != 0:
        raise ValueError("det F <= 0")
    return R


def fem_tet_eval(Dm_inv, x, R=None):
    """Corotational strain C[6] (xx, yy, zz, yz, xz, xy), Jacobian J[6][12]
    with the rotation held fixed, and the rotation R (given, or the polar
    one of F)."""
    Dm_inv, x = _d(Dm_inv), _d(x)
    Rm = np.zeros((3, 3)) if R is None else _d(R).copy()
    Cv, J = np.zeros(6), np.zeros((6, 12))
    if lib().fem_tet_eval(_ptr(Dm_inv), _ptr(x), _ptr(Rm), 0 if R is None else 1, _ptr(Cv), _ptr(J)) != 0:
        raise ValueError("inverted tetrahedron")
    return Cv, J, Rm


def fem_tet_compliance(V, Y, nu):
    E = np.zeros((6, 6))
    lib().fem_tet_compliance(float(V), float(Y), float(nu), _ptr(E))
    return E


def fem_expansion(p, Y):
    return lib().fem_expansion(float(p), float(Y))


def fem_dist(xi, xj, r, p, Y):
    """Actuation distance constraint value and Jacobian J[6] (xi, xj)."""
    xi, xj, J = _d(xi), _d(xj), np.zeros(6)
    c = lib().fem_dist_eval(_ptr(xi), _ptr(xj), float(r), float(p), float(Y), _ptr(J))
    return c, J


def fem_attach(x, q, r, xp):
    """Attachment constraint C[3] and Jacobian J[3][9] (body x, body
    rotation, particle)."""
    x, q, r, xp = _d(x), _d(q), _d(r), _d(xp)
    Cv, J = np.zeros(3), np.zeros((3, 9))
    lib().fem_attach_eval(_ptr(x), _ptr(q), _ptr(r), _ptr(xp), _ptr(Cv), _ptr(J))
    return Cv, J
