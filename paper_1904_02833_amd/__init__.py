"""Python binding of the MI355X snake solver (``libsnake.so``).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  PyTorch provides the device workspace and the stream.  The
library must have been built (``paper_1904_02833_amd.build.build()``);
loading fails loudly otherwise, there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SNAKE_SANITIZE=1 loads the host-sanitized build (CPU checks of the host
# paths only; its process preloads the sanitizer runtime)
LIB_PATH = os.path.join(HERE, "libsnake_san.so" if os.environ.get("SNAKE_SANITIZE") == "1" else "libsnake.so")

SIM_OK, SIM_EINVAL, SIM_ENOMEM, SIM_EDEVICE, SIM_ESTATE = 0, -1, -2, -3, -4
MEM_HOST, MEM_DEVICE = 0, 1
LAW_LAG, LAW_PAPER = 0, 1
CTRL_EXTERNAL, CTRL_SERPENOID, CTRL_SCHEDULE = 0, 1, 2
WARM_ZERO, WARM_PREV, WARM_MLP = 0, 1, 2
SOLVER_JACOBI, SOLVER_NEWTON, SOLVER_GS = 0, 1, 2
FLAG_FIXED_ROOT, FLAG_NO_GROUND, FLAG_WHEELS = 1, 2, 16
STATUS_NONFINITE, STATUS_NOT_CONVERGED, STATUS_FELL_BACK = 1, 2, 4

# state fields: bit -> (name, dtype, rows, length key)
FIELDS = [
    ("pos", np.float32, 3, "N"),
    ("quat", np.float32, 4, "N"),
    ("vel", np.float32, 3, "N"),
    ("angvel", np.float32, 3, "N"),
    ("pressure", np.float32, 2, "Mt"),
    ("lambda_joint", np.float32, 6, "J"),
    ("lambda_contact", np.float32, 3, "N"),
    ("cmd", np.float32, 1, "Mt"),
    ("residual", np.float32, 1, "n"),
    ("iters", np.int32, 1, "n"),
    ("status", np.int32, 1, "n"),
    ("step", np.int64, 1, "n"),
    ("iters_total", np.int64, 1, "n"),
    ("wheel_pos", np.float32, 3, "W2"),
    ("wheel_quat", np.float32, 4, "W2"),
    ("wheel_vel", np.float32, 3, "W2"),
    ("wheel_angvel", np.float32, 3, "W2"),
    ("lambda_wheel", np.float32, 9, "W2"),
]
WHEEL_FIELDS = ("wheel_pos", "wheel_quat", "wheel_vel", "wheel_angvel", "lambda_wheel")
FIELD_BIT = {f[0]: 1 << k for k, f in enumerate(FIELDS)}
INDEX = ["body_off", "joint_off", "module_off", "block_off", "blk_type", "blk_a", "blk_b",
         "blk_color", "degree", "bucket", "order"]
EXPORTS = ["sim_workspace_bytes", "sim_create", "sim_set_pressures", "sim_step",
           "sim_read_state", "sim_write_state", "sim_set_mlp", "sim_step_record", "sim_read_index",
           "sim_sizes", "sim_mapping", "sim_plan_tiles", "sim_destroy", "sim_last_error"]

_P = C.c_void_p


class Desc(C.Structure):
    _fields_ = [
        ("n_snakes", C.c_int32),
        ("n_modules", _P), ("segs_per_module", _P),
        ("alpha_stretch", _P), ("alpha_bend", _P), ("alpha_twist", _P), ("mu", _P),
        ("seg_mass", C.c_double), ("seg_length", C.c_double), ("seg_radius", C.c_double),
        ("gravity", C.c_double),
        ("dt", C.c_double), ("substeps", C.c_int32), ("iters", C.c_int32),
        ("tol", C.c_double), ("relax", C.c_double),
        ("pressure_law", C.c_int32),
        ("tau_inflate", C.c_double), ("tau_deflate", C.c_double), ("kappa_max", C.c_double),
        ("k_inflate", C.c_double), ("k_deflate", C.c_double), ("T_p", C.c_double),
        ("p_source", C.c_double), ("amplitude_psi", C.c_double),
        ("controller", C.c_int32),
        ("ctrl_freq", _P), ("ctrl_phase0", _P),
        ("ctrl_alpha", C.c_double), ("ctrl_offset", C.c_double),
        ("sched_off", _P), ("sched_steps", _P), ("sched_val", _P),
        ("warm_start", C.c_int32), ("flags", C.c_uint32), ("use_graph", C.c_int32),
        ("autotune", C.c_int32), ("map_waves", C.c_int32), ("map_min_seg", C.c_int32),
        ("map_grid", C.c_int32), ("mlp_fallback", C.c_int32), ("map_rows", C.c_int32),
        ("mlp_fallback_k", C.c_int32), ("solver", C.c_int32), ("newton_iters", C.c_int32),
        ("pcr_iters", C.c_int32), ("newton_keep_best", C.c_int32),
    ]


_lib = None


def lib():
    """Load libsnake.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1904_02833_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        L.sim_workspace_bytes.argtypes = [C.POINTER(Desc), C.POINTER(C.c_size_t)]
        L.sim_create.argtypes = [C.POINTER(Desc), _P, C.c_size_t, _P, C.POINTER(_P)]
        L.sim_set_pressures.argtypes = [_P, _P, C.c_int64, C.c_int]
        L.sim_step.argtypes = [_P, C.c_int32]
        L.sim_read_state.argtypes = [_P, C.c_uint32, C.POINTER(_P), C.c_int]
        L.sim_write_state.argtypes = [_P, C.c_uint32, C.POINTER(_P), C.c_int]
        L.sim_read_index.argtypes = [_P, C.c_int32, _P, C.c_int64]
        L.sim_sizes.argtypes = [_P, C.POINTER(C.c_int64)]
        L.sim_mapping.argtypes = [_P, C.POINTER(C.c_int32)]
        L.sim_plan_tiles.argtypes = [C.POINTER(Desc), C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.sim_set_mlp.argtypes = [_P, _P, _P, C.c_int]
        L.sim_step_record.argtypes = [_P, C.c_int32, _P, _P, C.c_int64, C.POINTER(C.c_int64)]
        L.sim_destroy.argtypes = [_P]
        L.sim_destroy.restype = None
        L.sim_last_error.argtypes = []
        L.sim_last_error.restype = C.c_char_p
        _lib = L
    return _lib


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _check(rc):
    if rc != SIM_OK:
        raise SimError(rc, lib().sim_last_error().decode())


def _arr(keep, a, dt):
    a = np.ascontiguousarray(np.asarray(a, dtype=dt))
    keep.append(a)
    return a.ctypes.data_as(_P)


def make_desc(wl, **over):
    """sim_desc_t from a workload (any object with the workload fields);
    keyword overrides replace fields.  Returns (desc, keep-alive list)."""
    g = lambda k: over.get(k, getattr(wl, k))  # noqa: E731
    keep = []
    d = Desc()
    d.n_snakes = int(len(g("n_modules")))
    d.n_modules = _arr(keep, g("n_modules"), np.int32)
    d.segs_per_module = _arr(keep, g("segs_per_module"), np.int32)
    d.alpha_stretch = _arr(keep, g("alpha_stretch"), np.float64)
    d.alpha_bend = _arr(keep, g("alpha_bend"), np.float64)
    d.alpha_twist = _arr(keep, g("alpha_twist"), np.float64)
    d.mu = _arr(keep, g("mu"), np.float64)
    for f in ("seg_mass", "seg_length", "seg_radius", "gravity", "dt", "tol", "relax",
              "tau_inflate", "tau_deflate", "kappa_max", "k_inflate", "k_deflate", "T_p",
              "p_source", "amplitude_psi", "ctrl_alpha", "ctrl_offset"):
        setattr(d, f, float(g(f)))
    d.substeps = int(g("substeps"))
    d.iters = int(g("iters"))
    d.pressure_law = int(g("pressure_law"))
    d.controller = int(g("controller"))
    d.ctrl_freq = _arr(keep, g("ctrl_freq"), np.float64)
    d.ctrl_phase0 = _arr(keep, g("ctrl_phase0"), np.float64)
    if g("sched_off") is not None:
        d.sched_off = _arr(keep, g("sched_off"), np.int32)
        d.sched_steps = _arr(keep, g("sched_steps"), np.int32)
        d.sched_val = _arr(keep, g("sched_val"), np.float64)
    d.warm_start = int(over.get("warm_start", WARM_ZERO))
    d.flags = int(g("flags"))
    d.use_graph = int(over.get("use_graph", 1))
    d.autotune = int(over.get("autotune", 0))
    d.map_waves = int(over.get("map_waves", 0))
    d.map_min_seg = int(over.get("map_min_seg", 0))
    d.map_grid = int(over.get("map_grid", 0))
    d.mlp_fallback = int(over.get("mlp_fallback", 1))
    d.map_rows = int(over.get("map_rows", 0))
    d.mlp_fallback_k = int(over.get("mlp_fallback_k", 0))
    d.solver = int(over.get("solver", getattr(wl, "solver", SOLVER_JACOBI)))
    d.newton_iters = int(over.get("newton_iters", getattr(wl, "newton_iters", 4)))
    d.pcr_iters = int(over.get("pcr_iters", getattr(wl, "pcr_iters", 20)))
    d.newton_keep_best = int(over.get("newton_keep_best", 0))
    return d, keep


def plan_tiles(wl, waves, min_seg=16, rows=0, **over):
    """Host-side tile plan (no device): (hdr [tiles, 4], slots [n, 2]) int32,
    as described with sim_plan_tiles in include/snake.h."""
    L = lib()
    d, keep = make_desc(wl, **over)
    n = d.n_snakes
    hdr = np.zeros((n, 4), np.int32)
    slots = np.zeros((n, 2), np.int32)
    nt = C.c_int64(0)
    _check(L.sim_plan_tiles(C.byref(d), int(waves), int(min_seg), int(rows),
                            hdr.ctypes.data_as(C.POINTER(C.c_int32)), slots.ctypes.data_as(C.POINTER(C.c_int32)),
                            C.byref(nt)))
    del keep
    return hdr[:nt.value].copy(), slots


def workspace_bytes(wl, **over) -> int:
    d, _keep = make_desc(wl, **over)
    n = C.c_size_t(0)
    _check(lib().sim_workspace_bytes(C.byref(d), C.byref(n)))
    return int(n.value)


class Sim:
    """One batched solver on a GPU.  ``wl`` is a workload; keyword
    overrides replace its fields (``warm_start``, ``use_graph`` too)."""

    def __init__(self, wl, device="cuda", stream=None, **over):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the snake solver needs a ROCm GPU; none is visible")
        self.L = lib()
        self.torch = torch
        self.device = torch.device(device)
        d, keep = make_desc(wl, **over)
        n = C.c_size_t(0)
        _check(self.L.sim_workspace_bytes(C.byref(d), C.byref(n)))
        self.ws_bytes = int(n.value)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = (self.ws.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _P()
        _check(self.L.sim_create(C.byref(d), _P(base), self.ws_bytes, _P(self.stream.cuda_stream),
                                 C.byref(h)))
        self.h = h
        sz = (C.c_int64 * 5)()
        _check(self.L.sim_sizes(self.h, sz))
        self.n, self.N, self.J, self.Mt, self.n_blocks = (int(v) for v in sz)
        mp = (C.c_int32 * 5)()
        _check(self.L.sim_mapping(self.h, mp))
        self.mapping = dict(waves=mp[0], min_seg=mp[1], grid=mp[2], tiles=mp[3], rows=mp[4])
        self._substeps = d.substeps
        self._len = dict(n=self.n, N=self.N, J=self.J, Mt=self.Mt, W2=2 * self.N)
        self.wheels = bool(d.flags & FLAG_WHEELS)
        del keep

    def __del__(self):
        self.close()

    def close(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.L.sim_destroy(h)
            self.h = None

    # -- calls -------------------------------------------------------------
    def step(self, n_steps: int = 1):
        _check(self.L.sim_step(self.h, int(n_steps)))

    def set_pressures(self, cmd):
        """Commands, one per module: numpy (host) or a device tensor."""
        if hasattr(cmd, "is_cuda") and cmd.is_cuda:
            t = cmd.to(self.torch.float32).contiguous()
            _check(self.L.sim_set_pressures(self.h, _P(t.data_ptr()), t.numel(), MEM_DEVICE))
            self._cmd_keep = t
        else:
            a = np.ascontiguousarray(np.asarray(cmd, np.float32))
            _check(self.L.sim_set_pressures(self.h, a.ctypes.data_as(_P), a.size, MEM_HOST))

    def _shape(self, k):
        name, dt, rows, key = FIELDS[k]
        ln = self._len[key]
        return (rows, ln) if rows > 1 else (ln,)

    def read(self, *names) -> dict:
        """Host copies of the named fields (all if none), SoA as stored."""
        names = names or tuple(f[0] for f in FIELDS if self.wheels or f[0] not in WHEEL_FIELDS)
        ptrs = (_P * len(FIELDS))()
        out, mask = {}, 0
        for name in names:
            k = [f[0] for f in FIELDS].index(name)
            a = np.empty(self._shape(k), FIELDS[k][1])
            out[name] = a
            ptrs[k] = a.ctypes.data_as(_P)
            mask |= 1 << k
        _check(self.L.sim_read_state(self.h, mask, ptrs, MEM_HOST))
        return out

    def write(self, **fields):
        ptrs = (_P * len(FIELDS))()
        keep, mask = [], 0
        for name, val in fields.items():
            k = [f[0] for f in FIELDS].index(name)
            a = np.ascontiguousarray(np.asarray(val, FIELDS[k][1]).reshape(self._shape(k)))
            keep.append(a)
            ptrs[k] = a.ctypes.data_as(_P)
            mask |= 1 << k
        _check(self.L.sim_write_state(self.h, mask, ptrs, MEM_HOST))

    def read_device(self, names, tensors):
        """Device-to-device copies into torch tensors (same layouts)."""
        ptrs = (_P * len(FIELDS))()
        mask = 0
        for name, t in zip(names, tensors):
            k = [f[0] for f in FIELDS].index(name)
            ptrs[k] = _P(t.data_ptr())
            mask |= 1 << k
        _check(self.L.sim_read_state(self.h, mask, ptrs, MEM_DEVICE))

    def set_mlp(self, params, mean_std):
        """Network parameters and normalisation, torch device tensors."""
        p = params.to(self.torch.float32).contiguous()
        ms = mean_std.to(self.torch.float32).contiguous()
        _check(self.L.sim_set_mlp(self.h, _P(p.data_ptr()), _P(ms.data_ptr()), MEM_DEVICE))
        self._mlp_keep = (p, ms)

    def step_record(self, n_steps, features, targets):
        """Advance and record network inputs / targets into device tensors
        features[rows, 32], targets[rows, 3]; returns the rows written."""
        w = C.c_int64(0)
        _check(self.L.sim_step_record(self.h, int(n_steps), _P(features.data_ptr()),
                                      _P(targets.data_ptr()), features.shape[0], C.byref(w)))
        return int(w.value)

    def record_rows(self, n_steps):
        return 2 * self.J * int(self._substeps) * int(n_steps)

    def index(self, name) -> np.ndarray:
        k = INDEX.index(name)
        ln = {"body_off": self.n + 1, "joint_off": self.n + 1, "module_off": self.n + 1,
              "block_off": self.n + 1, "degree": self.N, "bucket": self.n,
              "order": self.n}.get(name, self.n_blocks)
        a = np.empty(ln, np.int32)
        _check(self.L.sim_read_index(self.h, k, a.ctypes.data_as(_P), ln))
        return a


# ---------------------------------------------------------------- network

MLP_EXPORTS = ["mlp_param_count", "mlp_train_scratch_floats", "mlp_norm_stats", "mlp_forward",
               "mlp_grad", "mlp_grad_noalloc", "mlp_adam", "mlp_last_error"]


def _mlp_lib():
    L = lib()
    if not getattr(L, "_mlp_declared", False):
        L.mlp_param_count.restype = C.c_int
        L.mlp_train_scratch_floats.argtypes = [C.c_int64]
        L.mlp_train_scratch_floats.restype = C.c_int64
        L.mlp_norm_stats.argtypes = [_P, C.c_int64, _P, _P]
        L.mlp_forward.argtypes = [_P, _P, _P, _P, C.c_int64, _P]
        L.mlp_grad.argtypes = [_P, _P, _P, _P, C.c_int64, _P, _P, _P, C.c_int64, _P]
        L.mlp_grad_noalloc.argtypes = [_P, _P, _P, _P, C.c_int64, _P, _P, _P]
        L.mlp_adam.argtypes = [_P, _P, _P, _P, C.c_int32, C.c_float, _P]
        L.mlp_last_error.restype = C.c_char_p
        L._mlp_declared = True
    return L


def _mcheck(rc):
    if rc != SIM_OK:
        raise SimError(rc, _mlp_lib().mlp_last_error().decode())


def _dp(t):
    assert t.is_cuda and t.is_contiguous() and t.dtype.is_floating_point
    return _P(t.data_ptr())


def _stream(t):
    import torch
    return _P(torch.cuda.current_stream(t.device).cuda_stream)


class Net:
    """Device-resident warm-start network: FP32 parameters, normalisation
    statistics and Adam state in torch tensors; every operation runs in the
    library's kernels."""

    def __init__(self, params, mean_std, device="cuda"):
        import torch
        self.torch = torch
        self.P = int(_mlp_lib().mlp_param_count())
        self.params = torch.as_tensor(params, dtype=torch.float32, device=device).contiguous()
        self.mean_std = torch.as_tensor(mean_std, dtype=torch.float32, device=device).contiguous()
        assert self.params.numel() == self.P and self.mean_std.numel() == 64
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self._scratch = None

    @staticmethod
    def norm_stats(x):
        import torch
        ms = torch.empty(64, dtype=torch.float32, device=x.device)
        _mcheck(_mlp_lib().mlp_norm_stats(_dp(x), x.shape[0], _dp(ms), _stream(x)))
        return ms

    def forward(self, x):
        y = self.torch.empty((x.shape[0], 3), dtype=self.torch.float32, device=x.device)
        _mcheck(_mlp_lib().mlp_forward(_dp(self.params), _dp(self.mean_std), _dp(x), _dp(y),
                                       x.shape[0], _stream(x)))
        return y

    def grad(self, x, t):
        L = _mlp_lib()
        need = int(L.mlp_train_scratch_floats(x.shape[0]))
        if self._scratch is None or self._scratch.numel() < need:
            self._scratch = self.torch.empty(need, dtype=self.torch.float32, device=x.device)
        g = self.torch.empty_like(self.params)
        loss = self.torch.empty(1, dtype=self.torch.float32, device=x.device)
        _mcheck(L.mlp_grad(_dp(self.params), _dp(self.mean_std), _dp(x), _dp(t), x.shape[0], _dp(g),
                           _dp(loss), _dp(self._scratch), self._scratch.numel(), _stream(x)))
        return g, loss

    def grad_noalloc(self, x, t):
        """mlp_grad through the entry point that allocates nothing (fixed
        library scratch, batches of at most 4096 samples)."""
        g = self.torch.empty_like(self.params)
        loss = self.torch.empty(1, dtype=self.torch.float32, device=x.device)
        _mcheck(_mlp_lib().mlp_grad_noalloc(_dp(self.params), _dp(self.mean_std), _dp(x), _dp(t), x.shape[0],
                                            _dp(g), _dp(loss), _stream(x)))
        return g, loss

    def adam(self, g, lr=1e-3):
        self.t += 1
        _mcheck(_mlp_lib().mlp_adam(_dp(self.params), _dp(self.m), _dp(self.v), _dp(g), self.t,
                                    float(lr), _stream(g)))
