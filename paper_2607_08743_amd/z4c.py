"""Python binding of libz4c.so (include/z4c.h): argument marshalling only.

Every step of the evolution runs in the HIP kernels of the library; this
module converts torch tensors (device memory, owned by the caller) and the
current HIP stream into the C arguments and turns error codes into
exceptions.  If the library is not built, every call raises: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

from . import inputs as _inputs

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libz4c.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "z4c.h")

NF = 25
OK, EINVAL, EHIP, ENOMEM, EUNSUPPORTED = 0, -1, -2, -3, -4
TILE_DEFAULT, TILE_CALLER, TILE_CACHE, TILE_TUNED = 0, 1, 2, 3
TILE_SOURCE_NAMES = {TILE_DEFAULT: "default", TILE_CALLER: "caller", TILE_CACHE: "cache", TILE_TUNED: "tuned"}
BC_PERIODIC, BC_SOMMERFELD, BC_COPY, BC_EQUATORIAL = 0, 1, 2, 3
FP64, MIXED = 0, 1


class Z4cError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("kappa1", ctypes.c_double), ("kappa2", ctypes.c_double), ("kappa3", ctypes.c_double),
                ("eta", ctypes.c_double), ("shift_coeff", ctypes.c_double), ("ko_sigma", ctypes.c_double),
                ("w_floor", ctypes.c_double), ("lapse_uses_K", ctypes.c_int), ("precision", ctypes.c_int)]


class Tile(ctypes.Structure):
    _fields_ = [("bx", ctypes.c_int), ("by", ctypes.c_int), ("bz", ctypes.c_int), ("waves", ctypes.c_int),
                ("persistent", ctypes.c_int)]

    def as_tuple(self):
        return (self.bx, self.by, self.bz, self.waves, self.persistent)


class Box(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("ng", ctypes.c_int), ("bc", ctypes.c_int), ("sf", ctypes.c_long),
                ("dx", ctypes.c_double * 3), ("x0", ctypes.c_double * 3), ("dt", ctypes.c_double),
                ("u_n", ctypes.c_void_p), ("u_a", ctypes.c_void_p), ("u_b", ctypes.c_void_p),
                ("acc", ctypes.c_void_p), ("shell", ctypes.c_void_p)]


class Level(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("ng", ctypes.c_int), ("bc", ctypes.c_int), ("sf", ctypes.c_long),
                ("dx", ctypes.c_double * 3), ("x0", ctypes.c_double * 3), ("F", ctypes.c_int * 3),
                ("u", ctypes.c_void_p), ("u_a", ctypes.c_void_p), ("u_b", ctypes.c_void_p),
                ("acc", ctypes.c_void_p), ("prev", ctypes.c_void_p), ("cur", ctypes.c_void_p),
                ("parent", ctypes.c_int), ("obj", ctypes.c_int)]


_lib = None


def lib(path: str = LIB_PATH):
    """Load libz4c.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libz4c.so is not built ({path}); run __graft_entry__.build() "
                           "or python -m paper_2607_08743_amd.build")
    # The library must run on the HIP runtime that owns torch's device memory
    # and streams.  torch ships its own libamdhip64; once it is loaded, the
    # library's dependency resolves to it by soname.  Loaded first, the
    # library would pull in a second, separate HIP runtime, in which torch's
    # stream handles are invalid (and which may not see the device at all).
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp, dp, i, l, d = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_double
    pp = ctypes.POINTER(Params)
    geo = [l, i, i, i, i, d, d, d, d, d, d, i]
    L.z4c_default_params.argtypes = [pp]
    L.z4c_default_params.restype = None
    L.rhs_z4c.argtypes = [dp, dp] + geo + [pp, vp]
    L.rk4_substep.argtypes = [i, d, dp, dp, dp, dp] + geo + [pp, vp]
    L.rk4_substep_monitor.argtypes = [i, d, dp, dp, dp, dp] + geo + [pp, dp, dp, dp, l, vp]
    L.z4c_monitor_workspace.argtypes = [i, i, i]
    L.z4c_monitor_workspace.restype = l
    L.apply_ghosts.argtypes = [dp, dp, l, i, i, i, i, i, vp]
    L.z4c_tile_count.argtypes = [i]
    L.z4c_tile_get.argtypes = [i, i, ctypes.POINTER(Tile)]
    L.z4c_select_tile.argtypes = [i, ctypes.POINTER(Tile)]
    L.z4c_tile_resources.argtypes = [i, ctypes.POINTER(Tile), ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]
    L.z4c_plan_create.argtypes = [ctypes.POINTER(Box), i, pp, ctypes.POINTER(Tile), ctypes.c_char_p,
                                  ctypes.POINTER(vp)]
    L.z4c_plan_tile.argtypes = [vp, ctypes.POINTER(Tile), ctypes.POINTER(i)]
    L.z4c_autotune.argtypes = [ctypes.POINTER(Box), i, pp, ctypes.c_char_p, vp, ctypes.POINTER(Tile),
                               ctypes.POINTER(i)]
    L.z4c_tune_lookup.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(Box), i, i,
                                  ctypes.POINTER(Tile)]
    L.z4c_plan_step.argtypes = [vp, i, i, vp]
    L.z4c_plan_autotune.argtypes = [vp, i, vp, ctypes.POINTER(Tile), ctypes.POINTER(ctypes.c_float)]
    L.z4c_plan_destroy.argtypes = [vp]
    L.z4c_hier_create.argtypes = [ctypes.POINTER(Level), i, pp, d, ctypes.POINTER(Tile), ctypes.POINTER(vp)]
    L.z4c_hier_advance.argtypes = [vp, i, i, vp]
    L.z4c_hier_destroy.argtypes = [vp]
    L.z4c_hier_set_moving.argtypes = [vp, i, ctypes.POINTER(ctypes.c_double)]
    L.z4c_hier_puncture.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_double)]
    L.z4c_constraints_workspace.argtypes = [i, i, i]
    L.z4c_constraints_workspace.restype = l
    L.z4c_constraints.argtypes = [dp, dp, dp, dp, l, l, i, i, i, i, d, d, d, vp]
    L.z4c_constraints_noalloc.argtypes = [dp, dp, dp, l, i, i, i, i, d, d, d, vp]
    L.z4c_strerror.argtypes = [i]
    L.z4c_strerror.restype = ctypes.c_char_p
    L.z4c_last_error.argtypes = []
    L.z4c_last_error.restype = ctypes.c_char_p
    for name in ("rhs_z4c", "rk4_substep", "rk4_substep_monitor", "apply_ghosts", "z4c_tile_count", "z4c_tile_get", "z4c_select_tile",
                 "z4c_tile_resources",
                 "z4c_plan_create", "z4c_plan_step", "z4c_plan_autotune", "z4c_plan_destroy", "z4c_constraints",
                 "z4c_plan_tile", "z4c_autotune", "z4c_tune_lookup", "z4c_constraints_noalloc",
                 "z4c_hier_create", "z4c_hier_advance", "z4c_hier_destroy", "z4c_hier_set_moving", "z4c_hier_puncture"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/z4c.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int|long|void|char\s*\*|const char\s*\*)\s*\**\s*(\w+)\s*\(",
                                 text, flags=re.M)))


def check(status: int, where: str):
    if status != OK:
        L = lib()
        raise Z4cError(status, where, L.z4c_last_error().decode())


def default_params(**kw) -> Params:
    p = Params()
    lib().z4c_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _state_tensor(t, g, name):
    import torch
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if tuple(t.shape) != tuple(g.shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(g.shape)}")


def _geo(g, sf):
    return (ctypes.c_long(sf), int(g.n[0]), int(g.n[1]), int(g.n[2]), int(g.ng), float(g.h[0]), float(g.h[1]),
            float(g.h[2]), float(g.x0[0]), float(g.x0[1]), float(g.x0[2]), int(g.bc))


def rhs_z4c(u, rhs, g: _inputs.Grid, params: Params = None, stream=None):
    _state_tensor(u, g, "u")
    _state_tensor(rhs, g, "rhs")
    p = params or default_params()
    check(lib().rhs_z4c(_ptr(u), _ptr(rhs), *_geo(g, g.stored), ctypes.byref(p), _stream(stream)), "rhs_z4c")


def rk4_substep(stage, dt, u_in, u_n, acc, u_out, g: _inputs.Grid, params: Params = None, stream=None):
    for t, nm in ((u_in, "u_in"), (u_n, "u_n"), (acc, "acc"), (u_out, "u_out")):
        _state_tensor(t, g, nm)
    p = params or default_params()
    check(lib().rk4_substep(int(stage), float(dt), _ptr(u_in), _ptr(u_n), _ptr(acc), _ptr(u_out),
                            *_geo(g, g.stored), ctypes.byref(p), _stream(stream)), "rk4_substep")


def monitor_workspace(g: _inputs.Grid) -> int:
    """Doubles of device workspace rk4_substep_monitor needs for this box."""
    return int(lib().z4c_monitor_workspace(int(g.n[0]), int(g.n[1]), int(g.n[2])))


def rk4_substep_monitor(stage, dt, u_in, u_n, acc, u_out, g: _inputs.Grid, params: Params = None, c=None, norms=None,
                        ws=None, stream=None):
    """One float64 RK4 stage fused with the constraint monitor of u_in.
    Returns the (4,) tensor of L2 norms (H, M^x, M^y, M^z); c, if given, a
    (4, Nz, Ny, Nx) float64 CUDA tensor, receives the per-point values."""
    import torch
    for t, nm in ((u_in, "u_in"), (u_n, "u_n"), (acc, "acc"), (u_out, "u_out")):
        _state_tensor(t, g, nm)
    if c is not None and (c.dtype != torch.float64 or not c.is_cuda or not c.is_contiguous()
                          or tuple(c.shape) != (4,) + tuple(g.shape[1:])):
        raise TypeError("c must be a contiguous float64 CUDA tensor of shape (4, Nz, Ny, Nx)")
    p = params or default_params()
    if norms is None:
        norms = torch.empty(4, dtype=torch.float64, device=u_in.device)
    if ws is None:
        ws = torch.empty(max(monitor_workspace(g), 1), dtype=torch.float64, device=u_in.device)
    check(lib().rk4_substep_monitor(int(stage), float(dt), _ptr(u_in), _ptr(u_n), _ptr(acc), _ptr(u_out),
                                    *_geo(g, g.stored), ctypes.byref(p), _ptr(c), _ptr(norms), _ptr(ws),
                                    ctypes.c_long(ws.numel()), _stream(stream)), "rk4_substep_monitor")
    return norms


def apply_ghosts(u, g: _inputs.Grid, shell=None, stream=None):
    _state_tensor(u, g, "u")
    if shell is not None:
        import torch
        if shell.dtype != torch.float64 or not shell.is_cuda or not shell.is_contiguous():
            raise TypeError("shell must be a contiguous float64 CUDA tensor")
    check(lib().apply_ghosts(_ptr(u), _ptr(shell), ctypes.c_long(g.stored), int(g.n[0]), int(g.n[1]), int(g.n[2]),
                             int(g.ng), int(g.bc), _stream(stream)), "apply_ghosts")


def constraints_workspace(g: _inputs.Grid) -> int:
    """Doubles of device workspace z4c_constraints needs for this box."""
    return int(lib().z4c_constraints_workspace(int(g.n[0]), int(g.n[1]), int(g.n[2])))


def constraints(u, g: _inputs.Grid, c=None, norms=None, ws=None, stream=None):
    """Hamiltonian and momentum constraints of u (ghosts valid).  c: None or a
    (4, Nz, Ny, Nx) float64 CUDA tensor that receives H, M^x, M^y, M^z per
    point.  Returns the (4,) tensor of L2 norms (allocated here unless given,
    like the workspace)."""
    import torch
    _state_tensor(u, g, "u")
    if c is not None and (c.dtype != torch.float64 or not c.is_cuda or not c.is_contiguous()
                          or tuple(c.shape) != (4,) + tuple(g.shape[1:])):
        raise TypeError("c must be a contiguous float64 CUDA tensor of shape (4, Nz, Ny, Nx)")
    if norms is None:
        norms = torch.empty(4, dtype=torch.float64, device=u.device)
    nws = constraints_workspace(g)
    if ws is None:
        ws = torch.empty(max(nws, 1), dtype=torch.float64, device=u.device)
    check(lib().z4c_constraints(_ptr(u), _ptr(c), _ptr(norms), _ptr(ws), ctypes.c_long(ws.numel()),
                                ctypes.c_long(g.stored), int(g.n[0]), int(g.n[1]), int(g.n[2]), int(g.ng),
                                float(g.h[0]), float(g.h[1]), float(g.h[2]), _stream(stream)), "z4c_constraints")
    return norms


def constraints_noalloc(u, g: _inputs.Grid, c=None, norms=None, stream=None):
    """z4c_constraints_noalloc: the constraint monitor with the library's own
    fixed device array for the block sums (no workspace, nothing allocated by
    the library).  norms: a (4,) float64 CUDA tensor (allocated here if not
    given)."""
    import torch
    _state_tensor(u, g, "u")
    if c is not None and (c.dtype != torch.float64 or not c.is_cuda or not c.is_contiguous()
                          or tuple(c.shape) != (4,) + tuple(g.shape[1:])):
        raise TypeError("c must be a contiguous float64 CUDA tensor of shape (4, Nz, Ny, Nx)")
    if norms is None:
        norms = torch.empty(4, dtype=torch.float64, device=u.device)
    check(lib().z4c_constraints_noalloc(_ptr(u), _ptr(c), _ptr(norms), ctypes.c_long(g.stored), int(g.n[0]),
                                        int(g.n[1]), int(g.n[2]), int(g.ng), float(g.h[0]), float(g.h[1]),
                                        float(g.h[2]), _stream(stream)), "z4c_constraints_noalloc")
    return norms


def tiles(precision: int = FP64):
    L = lib()
    out = []
    for k in range(L.z4c_tile_count(precision)):
        t = Tile()
        check(L.z4c_tile_get(precision, k, ctypes.byref(t)), "z4c_tile_get")
        out.append(t)
    return out


def select_tile(precision: int, tile: Tile = None):
    check(lib().z4c_select_tile(precision, None if tile is None else ctypes.byref(tile)), "z4c_select_tile")


def tile_resources(precision: int, tile: Tile) -> dict:
    """z4c_tile_resources: occupancy (resident waves per SIMD), static LDS
    bytes per block and scratch bytes per lane of a compiled tile shape."""
    w, s, x = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(lib().z4c_tile_resources(precision, ctypes.byref(tile), ctypes.byref(w), ctypes.byref(s), ctypes.byref(x)),
          "z4c_tile_resources")
    return {"waves_per_simd": w.value, "lds_bytes": s.value, "scratch_bytes_per_lane": x.value}


class Stepper:
    """Owns the four state-sized device arrays of one box (u_n, two stage
    states, accumulator) and advances u_n with the single-box entry points:
    per RK4 substep one apply_ghosts and one rk4_substep call."""

    def __init__(self, g: _inputs.Grid, u0, dt: float, params: Params = None, shell=None, device="cuda"):
        import torch
        self.g, self.dt = g, float(dt)
        self.params = params or default_params()
        self.u = torch.as_tensor(u0, dtype=torch.float64, device=device).contiguous().clone()
        self.a = torch.empty_like(self.u)
        self.b = torch.empty_like(self.u)
        self.acc = torch.empty_like(self.u)
        self.shell = None if shell is None else torch.as_tensor(shell, dtype=torch.float64, device=device).contiguous()

    def step(self, nsteps: int = 1, stream=None):
        seq = ((self.u, self.a), (self.a, self.b), (self.b, self.a), (self.a, self.u))
        for _ in range(nsteps):
            for s, (src, dst) in enumerate(seq, start=1):
                apply_ghosts(src, self.g, self.shell, stream)
                rk4_substep(s, self.dt, src, self.u, self.acc, dst, self.g, self.params, stream)
        apply_ghosts(self.u, self.g, self.shell, stream)


def _device_boxes(boxes, device):
    """Device arrays (state copied in, three scratch arrays, shell) and the
    z4c_box array of a list of inputs.Box."""
    import torch
    us, keep, cboxes = [], [], []
    for bx in boxes:
        g = bx.grid
        u = torch.as_tensor(bx.state, dtype=torch.float64, device=device).contiguous().clone()
        a, b, acc = torch.empty_like(u), torch.empty_like(u), torch.empty_like(u)
        sh = None if bx.shell is None else torch.as_tensor(bx.shell, dtype=torch.float64, device=device).contiguous()
        us.append(u)
        keep.append((a, b, acc, sh))
        c = Box()
        c.n[:] = [int(v) for v in g.n]
        c.ng, c.bc, c.sf = int(g.ng), int(g.bc), int(g.stored)
        c.dx[:] = [float(v) for v in g.h]
        c.x0[:] = [float(v) for v in g.x0]
        c.dt = float(bx.dt)
        c.u_n, c.u_a, c.u_b, c.acc = u.data_ptr(), a.data_ptr(), b.data_ptr(), acc.data_ptr()
        c.shell = None if sh is None else sh.data_ptr()
        cboxes.append(c)
    return us, keep, (Box * len(cboxes))(*cboxes)


def _path(p):
    return None if p is None else os.fsencode(p)


def autotune(boxes, params: Params = None, tune_cache=None, stream=None, device="cuda"):
    """z4c_autotune over copies of the boxes: (tile, source name).  A cache
    hit returns the cached shape without running anything; a miss times every
    compiled shape and, with tune_cache set, persists the fastest."""
    p = params or default_params()
    us, keep, cb = _device_boxes(boxes, device)
    best, src = Tile(), ctypes.c_int()
    check(lib().z4c_autotune(cb, len(boxes), ctypes.byref(p), _path(tune_cache), _stream(stream), ctypes.byref(best),
                             ctypes.byref(src)), "z4c_autotune")
    del us, keep
    return best, TILE_SOURCE_NAMES[src.value]


def tune_lookup(tune_cache, arch: str, grids, precision: int = FP64):
    """Host-only query of the tuning cache: the cached Tile for boxes of
    these grids (extents only) on `arch`, or None on a miss."""
    cb = (Box * len(grids))()
    for c, g in zip(cb, grids):
        c.n[:] = [int(v) for v in g.n]
    t = Tile()
    rc = lib().z4c_tune_lookup(_path(tune_cache), arch.encode(), cb, len(grids), int(precision), ctypes.byref(t))
    if rc < 0:
        check(rc, "z4c_tune_lookup")
    return t if rc == 1 else None


class Plan:
    """Batched form: every box in one fused launch per substep, one RK4 step
    captured as a HIP graph and replayed.  Owns the per-box device arrays.
    tile: the shape to launch; else the tuning cache tune_cache's entry for
    this workload, else the library default."""

    def __init__(self, boxes, params: Params = None, tile: Tile = None, device="cuda", tune_cache=None):
        self.params = params or default_params()
        self.boxes = list(boxes)
        self.u, self._keep, self._cboxes = _device_boxes(self.boxes, device)
        h = ctypes.c_void_p()
        check(lib().z4c_plan_create(self._cboxes, len(self.boxes), ctypes.byref(self.params),
                                    None if tile is None else ctypes.byref(tile), _path(tune_cache),
                                    ctypes.byref(h)), "z4c_plan_create")
        self._h = h

    def tile(self):
        """(Tile launched, source name: default / caller / cache / tuned)."""
        t, src = Tile(), ctypes.c_int()
        check(lib().z4c_plan_tile(self._h, ctypes.byref(t), ctypes.byref(src)), "z4c_plan_tile")
        return t, TILE_SOURCE_NAMES[src.value]

    def step(self, nsteps: int = 1, use_graph: bool = True, stream=None):
        check(lib().z4c_plan_step(self._h, int(nsteps), int(bool(use_graph)), _stream(stream)), "z4c_plan_step")

    def autotune(self, reps: int = 3, stream=None):
        n = 2 * lib().z4c_tile_count(self.params.precision)
        ms = (ctypes.c_float * n)()
        best = Tile()
        check(lib().z4c_plan_autotune(self._h, int(reps), _stream(stream), ctypes.byref(best), ms), "autotune")
        return best, list(ms)

    def close(self):
        if getattr(self, "_h", None):
            lib().z4c_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hierarchy:
    """Box-in-box hierarchy with Berger-Oliger subcycling: levels[q] = (grid,
    state, F) or (grid, state, F, parent, obj) for patch q, with F the parent
    active cell index of the patch's lower faces (ignored for the root),
    parent the index of its parent patch (default: the patch before it) and
    obj the tracked object it follows (default -1: fixed).  Owns the six
    device arrays of every patch; u[q] is patch q's state."""

    def __init__(self, levels, dt0: float, params: Params = None, tile: Tile = None, device="cuda"):
        import torch
        self.params = params or default_params()
        self.grids = [lv[0] for lv in levels]
        self.u, self._keep, cl = [], [], []
        self.nobj = 0
        for q, lv in enumerate(levels):
            g, state, F = lv[:3]
            parent = lv[3] if len(lv) > 3 and lv[3] is not None else q - 1
            obj = lv[4] if len(lv) > 4 else -1
            u = torch.as_tensor(state, dtype=torch.float64, device=device).contiguous().clone()
            extra = [torch.zeros_like(u) for _ in range(5)]
            self.u.append(u)
            self._keep.append(extra)
            c = Level()
            c.n[:] = [int(v) for v in g.n]
            c.ng, c.bc, c.sf = int(g.ng), int(g.bc), int(g.stored)
            c.dx[:] = [float(v) for v in g.h]
            c.x0[:] = [float(v) for v in g.x0]
            c.F[:] = [int(v) for v in F]
            c.u = u.data_ptr()
            c.u_a, c.u_b, c.acc, c.prev, c.cur = [t.data_ptr() for t in extra]
            c.parent, c.obj = int(parent), int(obj)
            cl.append(c)
        self._cl = (Level * len(cl))(*cl)
        h = ctypes.c_void_p()
        check(lib().z4c_hier_create(self._cl, len(cl), ctypes.byref(self.params), float(dt0),
                                    None if tile is None else ctypes.byref(tile), ctypes.byref(h)), "z4c_hier_create")
        self._h = h

    def advance(self, nsteps: int = 1, use_graph: bool = True, stream=None):
        check(lib().z4c_hier_advance(self._h, int(nsteps), int(bool(use_graph)), _stream(stream)), "z4c_hier_advance")

    def set_moving(self, xp):
        """The patches with obj >= 0 follow the punctures xp (one row of 3 per
        object; a single row may be flat)."""
        x = np.ascontiguousarray(np.array(xp, dtype=np.float64).reshape(-1, 3))
        self.nobj = len(x)
        check(lib().z4c_hier_set_moving(self._h, self.nobj, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
              "z4c_hier_set_moving")

    def puncture(self):
        """(punctures (nobj, 3), [F per patch], [x0 per patch])."""
        n = len(self.grids)
        x = np.zeros((max(self.nobj, 1), 3))
        F = (ctypes.c_int * (3 * n))()
        x0 = (ctypes.c_double * (3 * n))()
        check(lib().z4c_hier_puncture(self._h, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if self.nobj else None,
                                      F, x0), "z4c_hier_puncture")
        return (x[:self.nobj], [tuple(F[3 * q:3 * q + 3]) for q in range(n)],
                [tuple(x0[3 * q:3 * q + 3]) for q in range(n)])

    def close(self):
        if getattr(self, "_h", None):
            lib().z4c_hier_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
