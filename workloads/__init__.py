"""Seeded synthetic workloads for the snake solver.

This module only draws numbers and holds the fixed settings of each workload.
It contains none of the solver's arithmetic: no dynamics, no constraint
functions, no controller evaluation.  Both the FP64 oracle and the GPU
library consume the same ``Workload`` object, so they see identical inputs.

The random stream is SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), drawn on the host in a fixed
order per snake.  A uniform double is ``(z >> 11) * 2**-53``.

Workloads (the paper's own robot data is not available; these synthetic
batches stand in for it):

* ``single``   1 snake, 4 modules x 16 segments, serpenoid 0.5 Hz,
               module phase pi/2, mu 0.5, 600 steps, 4 substeps x 20 iters.
* ``uniform``  4096 copies of that geometry with per-snake compliance
               U[1e-6,1e-4], mu U[0.2,0.8], frequency U[0.2,1.0] Hz and
               phase U[0,2pi]; 1000 steps, 4 x 20.
* ``uneven``   16384 snakes, modules U{2..8}, segments U{8..32}, the same
               parameter draws, piecewise-constant commands in [0,1] held
               for U{6..60} steps (0.1 to 1 s at 60 Hz); 1000 steps, 4 x 20.
* ``stiff``    256 snakes x 8 modules x 128 segments, compliance
               U[1e-8,1e-6], mu 0.6, serpenoid with the uniform-batch draws,
               residual tolerance 1e-4 (at most 200 iterations), 500 steps.
* ``learned``  the uneven batch, used with the learned warm start.
* ``short``    4096 snakes of 2 modules x U{3,4} segments (6 or 8 bodies),
               the uneven batch's parameter draws and commands: chains short
               enough that the solve reaches residual 1e-4 within a few
               thousand iterations (a setting for the learned warm start;
               not one of the paper's configurations).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

MASK64 = (1 << 64) - 1

# constants of the generator (published SplitMix64 definition)
_GAMMA = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB

# controller and pressure-law kinds (shared vocabulary with the C ABI)
CTRL_EXTERNAL = 0
CTRL_SERPENOID = 1
CTRL_SCHEDULE = 2
LAW_LAG = 0
LAW_PAPER = 1

WORKLOAD_NAMES = ("single", "uniform", "uneven", "stiff", "learned", "short")


class SplitMix64:
    """Counter-based 64-bit generator; pure Python integers, exact."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + _GAMMA) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * _MIX1) & MASK64
        z = ((z ^ (z >> 27)) * _MIX2) & MASK64
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        u = (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)
        return lo + (hi - lo) * u

    def integer(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive), by multiply-shift."""
        span = hi - lo + 1
        return lo + ((self.next_u64() >> 32) * span >> 32)


@dataclasses.dataclass
class Workload:
    """Inputs of one batched run.  All arrays are host numpy arrays."""

    name: str
    seed: int
    n_modules: np.ndarray        # int32 [n_snakes]
    segs_per_module: np.ndarray  # int32 [n_snakes]
    alpha_stretch: np.ndarray    # float64 [n_snakes], compliance per unit length
    alpha_bend: np.ndarray       # float64 [n_snakes]
    alpha_twist: np.ndarray      # float64 [n_snakes]
    mu: np.ndarray               # float64 [n_snakes]
    # controller
    controller: int
    ctrl_freq: np.ndarray        # float64 [n_snakes], Hz
    ctrl_phase0: np.ndarray      # float64 [n_snakes], rad
    ctrl_alpha: float = math.pi / 2   # phase shift between modules, rad
    ctrl_offset: float = 0.0          # offset added before the clamp
    sched_off: np.ndarray | None = None    # int32 [total_modules+1]
    sched_steps: np.ndarray | None = None  # int32 [n_pieces], length in steps
    sched_val: np.ndarray | None = None    # float64 [n_pieces], command in [-1,1]
    # body and world constants
    seg_mass: float = 0.02
    seg_length: float = 0.01
    seg_radius: float = 0.01
    gravity: float = 9.81
    # time stepping
    dt: float = 1.0 / 60.0
    substeps: int = 4
    iters: int = 20
    tol: float = 0.0             # <= 0: fixed iteration count
    relax: float = 1.0
    n_steps: int = 600
    # chamber pressure model
    pressure_law: int = LAW_LAG
    tau_inflate: float = 0.1
    tau_deflate: float = 0.2
    kappa_max: float = 10.0      # rest curvature at full differential pressure, 1/m
    k_inflate: float = 0.23
    k_deflate: float = 0.23
    T_p: float = 0.68            # psi
    p_source: float = 8.0        # psi
    amplitude_psi: float = 8.0   # psi that a command of 1 stands for
    flags: int = 0

    @property
    def n_snakes(self) -> int:
        return int(self.n_modules.shape[0])

    @property
    def bodies(self) -> np.ndarray:
        return (self.n_modules.astype(np.int64) * self.segs_per_module).astype(np.int64)

    @property
    def total_bodies(self) -> int:
        return int(self.bodies.sum())

    @property
    def total_modules(self) -> int:
        return int(self.n_modules.sum())

    def take(self, idx) -> "Workload":
        """Sub-batch made of the given snakes (schedules re-indexed)."""
        idx = np.asarray(idx, dtype=np.int64)
        w = dataclasses.replace(self)
        for f in ("n_modules", "segs_per_module", "alpha_stretch", "alpha_bend",
                  "alpha_twist", "mu", "ctrl_freq", "ctrl_phase0"):
            setattr(w, f, np.ascontiguousarray(getattr(self, f)[idx]))
        if self.sched_off is not None:
            mod_off = np.concatenate([[0], np.cumsum(self.n_modules.astype(np.int64))])
            offs, steps, vals = [0], [], []
            for s in idx:
                for m in range(mod_off[s], mod_off[s + 1]):
                    a, b = self.sched_off[m], self.sched_off[m + 1]
                    steps.append(self.sched_steps[a:b])
                    vals.append(self.sched_val[a:b])
                    offs.append(offs[-1] + (b - a))
            w.sched_off = np.asarray(offs, dtype=np.int32)
            w.sched_steps = (np.concatenate(steps) if steps else np.zeros(0)).astype(np.int32)
            w.sched_val = (np.concatenate(vals) if vals else np.zeros(0)).astype(np.float64)
        return w


def _draw_params(rng: SplitMix64, lo: float, hi: float, per_snake_mu: bool, mu_fixed: float):
    a_s = rng.uniform(lo, hi)
    a_b = rng.uniform(lo, hi)
    a_t = rng.uniform(lo, hi)
    mu = rng.uniform(0.2, 0.8) if per_snake_mu else mu_fixed
    f = rng.uniform(0.2, 1.0)
    ph = rng.uniform(0.0, 2.0 * math.pi)
    return a_s, a_b, a_t, mu, f, ph


def make(name: str, seed: int | None = None, n_snakes: int | None = None) -> Workload:
    """Build a named workload.  ``n_snakes`` truncates the batch (same draws
    for the snakes that remain, since every snake draws in a fixed order)."""
    if name not in WORKLOAD_NAMES:
        raise ValueError(f"unknown workload {name!r}")
    if seed is None:
        seed = 1000 + WORKLOAD_NAMES.index(name)
    rng = SplitMix64(seed)
    if name == "single":
        a_s, a_b, a_t = (rng.uniform(1e-6, 1e-4) for _ in range(3))
        n = 1
        w = Workload(name, seed,
                     n_modules=np.full(n, 4, np.int32), segs_per_module=np.full(n, 16, np.int32),
                     alpha_stretch=np.array([a_s]), alpha_bend=np.array([a_b]),
                     alpha_twist=np.array([a_t]), mu=np.array([0.5]),
                     controller=CTRL_SERPENOID, ctrl_freq=np.array([0.5]),
                     ctrl_phase0=np.array([0.0]), n_steps=600)
    elif name in ("uniform", "stiff"):
        full = 4096 if name == "uniform" else 256
        n = full if n_snakes is None else int(n_snakes)
        lo, hi = (1e-6, 1e-4) if name == "uniform" else (1e-8, 1e-6)
        cols = [_draw_params(rng, lo, hi, name == "uniform", 0.6) for _ in range(n)]
        a = np.array(cols, dtype=np.float64).reshape(n, 6)
        M, S = (4, 16) if name == "uniform" else (8, 128)
        w = Workload(name, seed,
                     n_modules=np.full(n, M, np.int32), segs_per_module=np.full(n, S, np.int32),
                     alpha_stretch=a[:, 0].copy(), alpha_bend=a[:, 1].copy(),
                     alpha_twist=a[:, 2].copy(), mu=a[:, 3].copy(),
                     controller=CTRL_SERPENOID, ctrl_freq=a[:, 4].copy(),
                     ctrl_phase0=a[:, 5].copy(),
                     n_steps=1000 if name == "uniform" else 500)
        if name == "stiff":
            w.tol = 1e-4
            w.iters = 200
    else:  # uneven / learned / short
        n = (4096 if name == "short" else 16384) if n_snakes is None else int(n_snakes)
        Ms, Ss, rows, offs, steps, vals = [], [], [], [0], [], []
        horizon = 1000
        for _ in range(n):
            if name == "short":
                M = 2
                S = rng.integer(3, 4)
            else:
                M = rng.integer(2, 8)
                S = rng.integer(8, 32)
            Ms.append(M)
            Ss.append(S)
            rows.append(_draw_params(rng, 1e-6, 1e-4, True, 0.0))
            for _m in range(M):
                covered = 0
                while covered < horizon + 1:
                    k = rng.integer(6, 60)
                    steps.append(k)
                    vals.append(rng.uniform(0.0, 1.0))
                    covered += k
                offs.append(len(steps))
        a = np.array(rows, dtype=np.float64).reshape(n, 6)
        w = Workload(name, seed,
                     n_modules=np.array(Ms, np.int32), segs_per_module=np.array(Ss, np.int32),
                     alpha_stretch=a[:, 0].copy(), alpha_bend=a[:, 1].copy(),
                     alpha_twist=a[:, 2].copy(), mu=a[:, 3].copy(),
                     controller=CTRL_SCHEDULE, ctrl_freq=a[:, 4].copy(),
                     ctrl_phase0=a[:, 5].copy(),
                     sched_off=np.array(offs, np.int32), sched_steps=np.array(steps, np.int32),
                     sched_val=np.array(vals, np.float64), n_steps=horizon)
    if n_snakes is not None and w.n_snakes > n_snakes:
        w = w.take(np.arange(n_snakes))
    return w


def custom(n_modules, segs_per_module, *, alpha=(1e-5, 1e-5, 1e-5), mu=0.5,
           controller=CTRL_EXTERNAL, freq=0.5, phase0=0.0, **kw) -> Workload:
    """Hand-built batch for tests: per-snake geometry, shared parameters."""
    nm = np.atleast_1d(np.asarray(n_modules, np.int32))
    sp = np.atleast_1d(np.asarray(segs_per_module, np.int32))
    if sp.shape[0] == 1 and nm.shape[0] > 1:
        sp = np.full_like(nm, sp[0])
    n = nm.shape[0]

    def col(v):
        v = np.atleast_1d(np.asarray(v, np.float64))
        return np.full(n, v[0]) if v.shape[0] == 1 else v.copy()

    return Workload("custom", 0, n_modules=nm, segs_per_module=sp,
                    alpha_stretch=col(alpha[0]), alpha_bend=col(alpha[1]),
                    alpha_twist=col(alpha[2]), mu=col(mu), controller=controller,
                    ctrl_freq=col(freq), ctrl_phase0=col(phase0), **kw)


def link_mesh(sections: int = 13, ring: int = 8, length: float = 0.01, radius: float = 0.01):
    """Procedural tetrahedral mesh of one soft link, a stand-in for the
    paper's TetGen mesh (not distributed): `sections` cross-sections evenly
    along x in [0, length], each a centre particle and `ring` particles on a
    circle of `radius` (radially symmetric); between consecutive sections
    every wedge (centre, k, k+1) is split into three tetrahedra with the
    diagonals centre -> next section's ring on its radial faces and ring k ->
    next section's ring k+1 on its outer face, so neighbouring wedges share
    whole triangles.  Returns particles [n][3] (section-major: centre, then
    the ring) and positively oriented tetrahedra [m][4] (particle indices)."""
    per = ring + 1
    xs = np.linspace(0.0, length, sections)
    th = 2.0 * np.pi * np.arange(ring) / ring
    pts = []
    for x in xs:
        pts.append([x, 0.0, 0.0])
        for t in th:
            pts.append([x, radius * np.cos(t), radius * np.sin(t)])
    pts = np.array(pts)
    tets = []
    for s in range(sections - 1):
        for k in range(ring):
            a0, a1, a2 = s * per, s * per + 1 + k, s * per + 1 + (k + 1) % ring
            b0, b1, b2 = a0 + per, a1 + per, a2 + per
            for t in ((a0, a1, a2, b2), (a0, a1, b1, b2), (a0, b0, b1, b2)):
                p = pts[list(t)]
                if np.linalg.det((p[1:] - p[0]).T) < 0:
                    t = (t[0], t[2], t[1], t[3])
                tets.append(t)
    return pts, np.array(tets, np.int64)


@dataclasses.dataclass
class LinkWorkload:
    """A batch of snakes built from full-resolution soft links (a
    tetrahedral particle mesh per link, rigid frames at the junctions).
    Every snake has the same links; friction differs per snake.  Commands
    are external: `link_commands` draws them."""
    name: str
    seed: int
    n_links: int
    sections: int
    ring: int
    X: np.ndarray                # float64 [per_link][3] link mesh, link frame
    tets: np.ndarray             # int32 [n_tets][4]
    mu: np.ndarray               # float64 [n_snakes]
    link_length: float = 0.16    # 16 cm: four 1 cm segments' modules of the chain workloads
    radius: float = 0.01
    young: float = 66243.0       # Pa, Ecoflex 00-30 (section "Soft robotic snake model")
    poisson: float = 0.4999
    density: float = 1070.0      # kg/m^3 (not given in the paper)
    p_max: float = 5333.0        # Pa at full chamber pressure: eq. expansion then bends a link to 10 1/m
    frame_mass: float = 0.02
    frame_length: float = 0.01
    gravity: float = 9.81
    dt: float = 1.0 / 60.0
    substeps: int = 4
    iters: int = 20
    tol: float = 0.0
    relax: float = 1.0
    tau_inflate: float = 0.1
    tau_deflate: float = 0.2
    rigid_compliance: float = 1e-7   # m/N on the non-deformable distance rows and the attachments
    flags: int = 0

    @property
    def n_snakes(self) -> int:
        return int(self.mu.shape[0])

    @property
    def per_link(self) -> int:
        return self.sections * (self.ring + 1)

    @property
    def particles(self) -> int:
        """particles per snake"""
        return self.n_links * self.per_link

    @property
    def n_tets(self) -> int:
        """tetrahedra per link"""
        return int(self.tets.shape[0])

    def take(self, idx) -> "LinkWorkload":
        w = dataclasses.replace(self)
        w.mu = np.ascontiguousarray(self.mu[np.asarray(idx, np.int64)])
        return w


def make_link(n_snakes: int = 2048, n_links: int = 4, seed: int = 1006, sections: int = 13,
              ring: int = 8) -> LinkWorkload:
    """The link batch: `n_snakes` snakes of `n_links` links on the procedural
    13-section mesh (the paper's snake has four links), friction U[0.2, 0.8]
    per snake."""
    rng = SplitMix64(seed)
    mu = np.array([rng.uniform(0.2, 0.8) for _ in range(n_snakes)], np.float64)
    X, tets = link_mesh(sections, ring, length=0.16, radius=0.01)
    return LinkWorkload("link", seed, n_links, sections, ring, X, tets.astype(np.int32), mu)


def link_commands(wl: LinkWorkload, n_steps: int, seed: int | None = None) -> np.ndarray:
    """Piecewise-constant signed commands per link, U[-1, 1] held for
    U{6..60} steps: float64 [n_steps][n_snakes * n_links]."""
    rng = SplitMix64(wl.seed + 17 if seed is None else seed)
    n = wl.n_snakes * wl.n_links
    out = np.empty((n_steps, n), np.float64)
    for c in range(n):
        t = 0
        while t < n_steps:
            k = rng.integer(6, 60)
            out[t:t + k, c] = rng.uniform(-1.0, 1.0)
            t += k
    return out
