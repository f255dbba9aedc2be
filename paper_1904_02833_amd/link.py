"""Python binding of the full-resolution link solver (``link_*`` in
``libsnake.so``, include/link.h).  Argument marshalling only: every step of
the solve runs in the library's HIP kernels; torch provides the workspace
and the stream.  No CPU path."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lib as _snake_lib

_P = C.c_void_p
LINK_OK = 0
MEM_HOST, MEM_DEVICE = 0, 1
FLAG_FIXED_FRAME0, FLAG_NO_GROUND = 1, 2
STATUS_NONFINITE, STATUS_NOT_CONVERGED = 1, 2
EXPORTS = ["link_workspace_bytes", "link_create", "link_set_commands", "link_step", "link_read_state",
           "link_write_state", "link_read_index", "link_plan_gathers", "link_sizes", "link_destroy",
           "link_last_error"]
# state fields: bit -> (name, dtype, rows, length key)
FIELDS = [
    ("pos", np.float32, 3, "P"), ("vel", np.float32, 3, "P"),
    ("frame_pos", np.float32, 3, "F"), ("frame_quat", np.float32, 4, "F"),
    ("frame_vel", np.float32, 3, "F"), ("frame_angvel", np.float32, 3, "F"),
    ("pressure", np.float32, 2, "L"), ("cmd", np.float32, 1, "L"),
    ("lambda_tet", np.float32, 6, "T"), ("lambda_dist", np.float32, 1, "D"),
    ("lambda_att", np.float32, 3, "A"), ("lambda_contact", np.float32, 3, "P"),
    ("residual", np.float32, 1, "n"), ("iters", np.int32, 1, "n"), ("status", np.int32, 1, "n"),
    ("iters_total", np.int32, 1, "n"),
]
INDEX = ["dist_i", "dist_j", "dist_kind", "degree_particle", "degree_frame"]


class LinkDesc(C.Structure):
    _fields_ = [
        ("n_snakes", C.c_int32), ("n_links", C.c_int32), ("sections", C.c_int32), ("ring", C.c_int32),
        ("n_tets", C.c_int32), ("X", _P), ("tets", _P), ("mu", _P),
        ("link_length", C.c_double), ("radius", C.c_double), ("young", C.c_double), ("poisson", C.c_double),
        ("density", C.c_double), ("p_max", C.c_double), ("frame_mass", C.c_double),
        ("frame_length", C.c_double), ("gravity", C.c_double), ("dt", C.c_double),
        ("substeps", C.c_int32), ("iters", C.c_int32), ("tol", C.c_double), ("relax", C.c_double),
        ("tau_inflate", C.c_double), ("tau_deflate", C.c_double), ("rigid_compliance", C.c_double),
        ("flags", C.c_uint32),
    ]


_declared = False


def lib():
    global _declared
    L = _snake_lib()
    if not _declared:
        dp = C.POINTER(LinkDesc)
        L.link_workspace_bytes.argtypes = [dp, C.POINTER(C.c_size_t)]
        L.link_create.argtypes = [dp, _P, C.c_size_t, _P, C.POINTER(_P)]
        L.link_set_commands.argtypes = [_P, _P, C.c_int64, C.c_int]
        L.link_step.argtypes = [_P, C.c_int32]
        L.link_read_state.argtypes = [_P, C.c_uint32, C.POINTER(_P), C.c_int]
        L.link_write_state.argtypes = [_P, C.c_uint32, C.POINTER(_P), C.c_int]
        L.link_read_index.argtypes = [_P, C.c_int32, _P, C.c_int64]
        L.link_plan_gathers.argtypes = [dp, _P, C.POINTER(C.c_int32)]
        L.link_sizes.argtypes = [_P, C.POINTER(C.c_int64)]
        L.link_destroy.argtypes = [_P]
        L.link_destroy.restype = None
        L.link_last_error.argtypes = []
        L.link_last_error.restype = C.c_char_p
        _declared = True
    return L


class LinkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _check(rc):
    if rc != LINK_OK:
        raise LinkError(rc, lib().link_last_error().decode())


def make_desc(wl, **over):
    """Descriptor of a ``workloads.LinkWorkload``; keyword overrides replace
    its settings.  Returns the descriptor and the arrays it points into."""
    g = lambda k: over.get(k, getattr(wl, k))  # noqa: E731
    keep = [np.ascontiguousarray(np.asarray(g("X"), np.float64)),
            np.ascontiguousarray(np.asarray(g("tets"), np.int32)),
            np.ascontiguousarray(np.asarray(g("mu"), np.float64))]
    d = LinkDesc()
    d.n_snakes = keep[2].shape[0]
    d.n_links, d.sections, d.ring = int(g("n_links")), int(g("sections")), int(g("ring"))
    d.n_tets = keep[1].shape[0]
    d.X, d.tets, d.mu = (a.ctypes.data_as(_P) for a in keep)
    for f, k in (("link_length", "link_length"), ("radius", "radius"), ("young", "young"), ("poisson", "poisson"),
                 ("density", "density"), ("p_max", "p_max"), ("frame_mass", "frame_mass"),
                 ("frame_length", "frame_length"), ("gravity", "gravity"), ("dt", "dt"), ("tol", "tol"),
                 ("relax", "relax"), ("tau_inflate", "tau_inflate"), ("tau_deflate", "tau_deflate"),
                 ("rigid_compliance", "rigid_compliance")):
        setattr(d, f, float(g(k)))
    d.substeps, d.iters, d.flags = int(g("substeps")), int(g("iters")), int(g("flags"))
    return d, keep


def workspace_bytes(wl, **over) -> int:
    d, keep = make_desc(wl, **over)
    n = C.c_size_t(0)
    _check(lib().link_workspace_bytes(C.byref(d), C.byref(n)))
    return int(n.value)


def plan_gathers(wl, **over):
    """The kernel's lane plan of the particles' gathers (host only):
    per lane (particle, group size, first, end) with particle -1 for an
    idle lane, and the largest group."""
    d, keep = make_desc(wl, **over)
    out = np.zeros(2048, np.int32)
    gmax = C.c_int32(0)
    _check(lib().link_plan_gathers(C.byref(d), out.ctypes.data_as(_P), C.byref(gmax)))
    w0, w1 = out[:1024], out[1024:]
    part = np.where(w0 >= 0, w0 & 0xffff, -1)
    size = np.where(w0 >= 0, 1 << (w0 >> 16), 0)
    return part, size, w1 & 0xffff, w1 >> 16, int(gmax.value)


class LinkSim:
    """A batch of link snakes on a GPU (one workgroup per snake)."""

    def __init__(self, wl, device="cuda", stream=None, **over):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the link solver needs a ROCm GPU; none is visible")
        self.L = lib()
        self.torch = torch
        self.device = torch.device(device)
        d, keep = make_desc(wl, **over)
        n = C.c_size_t(0)
        _check(self.L.link_workspace_bytes(C.byref(d), C.byref(n)))
        self.ws_bytes = int(n.value)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = (self.ws.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _P()
        _check(self.L.link_create(C.byref(d), _P(base), self.ws_bytes, _P(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        sz = (C.c_int64 * 10)()
        _check(self.L.link_sizes(self.h, sz))
        self.n, self.P, self.F, self.T, self.D, self.A, self.links, self.P1, self.D1, self.A1 = (int(v) for v in sz)
        self._len = dict(n=self.n, P=self.P, F=self.F, T=self.T, D=self.D, A=self.A, L=self.n * self.links)
        del keep

    def __del__(self):
        self.close()

    def close(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.L.link_destroy(h)
            self.h = None

    def step(self, n_steps: int = 1):
        _check(self.L.link_step(self.h, int(n_steps)))

    def set_commands(self, cmd):
        """One signed command per link: numpy (host) or a device tensor."""
        if hasattr(cmd, "is_cuda") and cmd.is_cuda:
            t = cmd.to(self.torch.float32).contiguous()
            _check(self.L.link_set_commands(self.h, _P(t.data_ptr()), t.numel(), MEM_DEVICE))
            self._cmd_keep = t
        else:
            a = np.ascontiguousarray(np.asarray(cmd, np.float32))
            _check(self.L.link_set_commands(self.h, a.ctypes.data_as(_P), a.size, MEM_HOST))

    def _shape(self, k):
        _, _, rows, key = FIELDS[k]
        ln = self._len[key]
        return (rows, ln) if rows > 1 else (ln,)

    def read(self, *names) -> dict:
        names = names or tuple(f[0] for f in FIELDS)
        ptrs = (_P * len(FIELDS))()
        out, mask = {}, 0
        for name in names:
            k = [f[0] for f in FIELDS].index(name)
            a = np.empty(self._shape(k), FIELDS[k][1])
            out[name] = a
            ptrs[k] = a.ctypes.data_as(_P)
            mask |= 1 << k
        _check(self.L.link_read_state(self.h, mask, ptrs, MEM_HOST))
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
        _check(self.L.link_write_state(self.h, mask, ptrs, MEM_HOST))

    def index(self, name) -> np.ndarray:
        k = INDEX.index(name)
        ln = {"dist_i": self.D1, "dist_j": self.D1, "dist_kind": self.D1, "degree_particle": self.P1,
              "degree_frame": self.links + 1}[name]
        a = np.empty(ln, np.int32)
        _check(self.L.link_read_index(self.h, k, a.ctypes.data_as(_P), ln))
        return a
