"""Python handle on the FP64 oracle of the full-resolution soft link
(``link_oracle.c``).  TEST INFRASTRUCTURE ONLY, like the rest of this
folder: the tests, the smoke check and the benchmark's CPU leg use it; the
GPU library never does.

State arrays are array-of-structures, float64: particles ``x[P,3]``,
``v[P,3]``; frames ``fx[F,3]``, ``fq[F,4]`` (w,x,y,z), ``fv[F,3]``,
``fw[F,3]``; chamber pressures ``p[snakes*links,2]`` (fraction of full),
commands ``cmd[snakes*links]``; multipliers ``lam_tet[T,6]`` (Voigt strain
order), ``lam_dist[D]``, ``lam_att[A,3]``, ``lam_c[P,3]`` (normal,
tangential x, y).  P, F, T, D, A count the whole batch.
"""
from __future__ import annotations

import ctypes as C
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import _ptr, lib

FIXED_FRAME0 = 1
NO_GROUND = 2
LINEARISED = 8
KIND_CENTRE, KIND_RADIAL, KIND_CHAMBER0, KIND_CHAMBER1 = 0, 1, 2, 3

_P = C.c_void_p


class LinkBatch(C.Structure):
    _fields_ = [
        ("n_snakes", C.c_int32), ("n_links", C.c_int32),
        ("sections", C.c_int32), ("ring", C.c_int32), ("n_tets", C.c_int32),
        ("X", _P), ("tets", _P), ("mu", _P),
        ("link_length", C.c_double), ("radius", C.c_double),
        ("young", C.c_double), ("poisson", C.c_double), ("density", C.c_double), ("p_max", C.c_double),
        ("frame_mass", C.c_double), ("frame_length", C.c_double),
        ("gravity", C.c_double), ("dt", C.c_double),
        ("substeps", C.c_int32), ("iters", C.c_int32),
        ("tol", C.c_double), ("relax", C.c_double), ("tau_inf", C.c_double), ("tau_def", C.c_double),
        ("rigid_compliance", C.c_double), ("flags", C.c_int32),
    ]


class LinkState(C.Structure):
    _fields_ = [(n, _P) for n in ("x", "v", "fx", "fq", "fv", "fw", "p", "cmd", "lam_tet", "lam_dist",
                                  "lam_att", "lam_c", "residual", "iters", "status")]


_declared = False


def _lib():
    global _declared
    L = lib()
    if not _declared:
        bp, sp = C.POINTER(LinkBatch), C.POINTER(LinkState)
        L.lnk_sizes.argtypes = [bp, _P]
        L.lnk_init_state.argtypes = [bp, sp]
        L.lnk_run.argtypes = [bp, sp, C.c_int32, C.c_int32, C.c_int32]
        L.lnk_run.restype = C.c_int
        L.lnk_assemble.argtypes = [bp, _P, _P, _P, _P, _P, _P, _P, _P]
        L.lnk_assemble.restype = C.c_int
        L.lnk_predict.argtypes = [bp] + [_P] * 6
        L.lnk_index.argtypes = [bp] + [_P] * 5
        L.lnk_link_masses.argtypes = [bp, _P]
        L.lnk_link_masses.restype = C.c_int
        L.lnk_link_dists.argtypes = [bp] + [_P] * 4
        L.lnk_link_atts.argtypes = [bp, _P, _P]
        _declared = True
    return L


class LinkOracle:
    """An FP64 link batch built from a ``workloads.LinkWorkload``; keyword
    overrides replace its settings (e.g. flags, iters, tol, dt, substeps)."""

    def __init__(self, wl, **over):
        self.L = _lib()
        g = lambda k: over.get(k, getattr(wl, k))  # noqa: E731
        self._keep = {}

        def arr(name, a, dt):
            a = np.ascontiguousarray(np.asarray(a, dtype=dt))
            self._keep[name] = a
            return _ptr(a)

        b = LinkBatch()
        b.n_snakes = int(np.asarray(g("mu")).shape[0])
        b.n_links, b.sections, b.ring = int(g("n_links")), int(g("sections")), int(g("ring"))
        b.n_tets = int(np.asarray(g("tets")).shape[0])
        b.X = arr("X", g("X"), np.float64)
        b.tets = arr("tets", g("tets"), np.int32)
        b.mu = arr("mu", g("mu"), np.float64)
        for f, k in (("link_length", "link_length"), ("radius", "radius"), ("young", "young"),
                     ("poisson", "poisson"), ("density", "density"), ("p_max", "p_max"),
                     ("frame_mass", "frame_mass"), ("frame_length", "frame_length"), ("gravity", "gravity"),
                     ("dt", "dt"), ("tol", "tol"), ("relax", "relax"), ("tau_inf", "tau_inflate"),
                     ("tau_def", "tau_deflate"), ("rigid_compliance", "rigid_compliance")):
            setattr(b, f, float(g(k)))
        b.substeps, b.iters, b.flags = int(g("substeps")), int(g("iters")), int(g("flags"))
        self.batch = b
        self.n = b.n_snakes
        sz = np.zeros(5, np.int32)
        self.L.lnk_sizes(C.byref(b), _ptr(sz))
        self.P, self.F, self.T, self.D, self.A = (int(v) for v in sz)
        n = self.n
        self.x = np.zeros((n * self.P, 3))
        self.v = np.zeros((n * self.P, 3))
        self.fx = np.zeros((n * self.F, 3))
        self.fq = np.zeros((n * self.F, 4))
        self.fv = np.zeros((n * self.F, 3))
        self.fw = np.zeros((n * self.F, 3))
        self.p = np.zeros((n * b.n_links, 2))
        self.cmd = np.zeros(n * b.n_links)
        self.lam_tet = np.zeros((n * self.T, 6))
        self.lam_dist = np.zeros(n * self.D)
        self.lam_att = np.zeros((n * self.A, 3))
        self.lam_c = np.zeros((n * self.P, 3))
        self.residual = np.zeros(n)
        self.iters = np.zeros(n, np.int32)
        self.status = np.zeros(n, np.int32)
        self.L.lnk_init_state(C.byref(b), C.byref(self._state()))

    def _state(self):
        s = LinkState()
        for k in ("x", "v", "fx", "fq", "fv", "fw", "p", "cmd", "lam_tet", "lam_dist", "lam_att", "lam_c",
                  "residual", "iters", "status"):
            setattr(s, k, _ptr(getattr(self, k)))
        return s

    def run(self, n_steps=1, threads=1, snakes=None):
        """Advance every snake (or the given range [s0, s1)) by n_steps with
        the held commands; snakes split over `threads` host threads."""
        s0, s1 = (0, self.n) if snakes is None else snakes
        st = self._state()
        if threads <= 1 or s1 - s0 <= 1:
            self.L.lnk_run(C.byref(self.batch), C.byref(st), s0, s1, n_steps)
            return
        cuts = np.linspace(s0, s1, min(threads, s1 - s0) + 1).round().astype(int)
        with ThreadPoolExecutor(len(cuts) - 1) as ex:
            list(ex.map(lambda k: self.L.lnk_run(C.byref(self.batch), C.byref(st), int(cuts[k]),
                                                 int(cuts[k + 1]), n_steps), range(len(cuts) - 1)))

    def index(self):
        """Degrees of one snake's particles and frames; its distance
        constraints' particle pairs and kinds (snake-local, int32)."""
        b = self.batch
        dp = np.zeros(self.P, np.int32)
        df = np.zeros(self.F, np.int32)
        di = np.zeros(self.D, np.int32)
        dj = np.zeros(self.D, np.int32)
        dk = np.zeros(self.D, np.int32)
        self.L.lnk_index(C.byref(b), _ptr(dp), _ptr(df), _ptr(di), _ptr(dj), _ptr(dk))
        return dict(degree_particle=dp, degree_frame=df, dist_i=di, dist_j=dj, dist_kind=dk)

    def link_masses(self):
        m = np.zeros(self.batch.sections * (self.batch.ring + 1))
        assert self.L.lnk_link_masses(C.byref(self.batch), _ptr(m)) == 0
        return m

    def link_dists(self):
        nd = self.D // self.batch.n_links
        pi, pj, kind = (np.zeros(nd, np.int32) for _ in range(3))
        rest = np.zeros(nd)
        self.L.lnk_link_dists(C.byref(self.batch), _ptr(pi), _ptr(pj), _ptr(kind), _ptr(rest))
        return pi, pj, kind, rest

    def link_atts(self):
        na = self.A // self.batch.n_links
        part, side = np.zeros(na, np.int32), np.zeros(na, np.int32)
        self.L.lnk_link_atts(C.byref(self.batch), _ptr(part), _ptr(side))
        return part, side

    def assemble(self, x, fx, fq, p):
        """Dense compliant system of one snake at (x, fx, fq) with chamber
        pressures p[links,2] (every block active, contacts left out):
        C[m], J[m,n], W[n,n], E[m,m] (compliance / h^2)."""
        n = 3 * self.P + 6 * self.F
        m = 6 * self.T + self.D + 3 * self.A
        Cv, J, Wm, E = np.zeros(m), np.zeros((m, n)), np.zeros((n, n)), np.zeros((m, m))
        args = [np.ascontiguousarray(a, np.float64) for a in (x, fx, fq, p)]
        got = self.L.lnk_assemble(C.byref(self.batch), *[_ptr(a) for a in args], _ptr(Cv), _ptr(J), _ptr(Wm),
                                  _ptr(E))
        assert got == m
        return Cv, J, Wm, E

    def predict(self, x, v, fx, fq, fv, fw):
        """One substep's prediction of one snake on copies of its state."""
        out = [np.array(a, np.float64, copy=True, order="C") for a in (x, v, fx, fq, fv, fw)]
        self.L.lnk_predict(C.byref(self.batch), *[_ptr(a) for a in out])
        return dict(zip(("x", "v", "fx", "fq", "fv", "fw"), out))
