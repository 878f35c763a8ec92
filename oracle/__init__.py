"""Plain FP64 CPU oracle for the Z4c right-hand side + RK4 step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2607_08743_amd``) never imports it and shares no code with it: the C
source ``z4c_oracle.c`` is an independent, per-point transcription of the
equations (paper Sec. 2.1.1 variables and gauge, Sec. 2.2 discretisation,
Sec. 2.2.2 Sommerfeld condition) and of the readings listed in its header.

Pins (each one is a test under ``tests/`` that checks the oracle against
something other than itself):

* stencils: exact on low-degree polynomials, 4th-order convergence, KO grid-mode
  eigenvalue -64, upwind bias gives a dissipative (stable) symbol;
* flat space: every right-hand side is exactly 0.0 and the state is unchanged;
* Schwarzschild in Kerr-Schild coordinates (analytic, SymPy): the 17 geometric
  right-hand sides vanish at O(h^4); gauge rows match their closed forms;
* Brill-Lindquist: Hamiltonian constraint drives N[Theta] -> 0 at O(h^4), and
  N[Khat] matches -D^2 alpha = -2 psi^-8 |grad psi|^2 (Laplace-Beltrami);
* conformally-flat / general data: N[At] matches the ADM-derived trace-free
  W^2(-D_iD_j alpha + alpha R_ij) computed from the physical metric;
* linearised plane wave propagates one period at 4th order;
* Z4 damping: homogeneous Theta and Z modes decay at rates kappa1(2+kappa2) and
  kappa1 through the classical RK4 amplification polynomial;
* Sommerfeld: F(t-r)/r gives the exact time derivative at 2nd order;
* pi symmetry: symmetrised data stays bitwise symmetric;
* equatorial symmetry: a half box with the reflection boundary evolves
  bitwise like the upper half of the full, z-symmetric Sommerfeld box (whose
  evolution uses no reflection code), and its ghost fill matches the parity
  rule written out independently in the test.

* shift terms of the Gt equation on data with Gt != Gt_d and a shift: the
  right-hand side's shift-dependent part converges at 4th order to
  -d_j (L_beta gt^ij) plus the transport of Zt = (Gt - Gt_d)/2 (advection
  for kappa3 = 0, the full Lie derivative of the density for kappa3 = 1),
  differentiated exactly: this pins the computed Gamma_d in the
  Lie-derivative terms and the kappa3 terms.

* the lapse trace: with zero shift, lapse_uses_K = 1 keeps alpha - ln det
  gamma constant (d_t alpha = tr(gamma^-1 d_t gamma) from the ADM metric
  evolution) on data with Theta != 0; the default (Khat) exceeds that by
  4 alpha Theta.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "z4c_oracle.c")
LIB = os.path.join(HERE, "liboracle_z4c.so")

NF = 25
BC_PERIODIC, BC_SOMMERFELD, BC_COPY, BC_EQUATORIAL = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class OzLevel(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("prev", ctypes.c_void_p), ("sf", ctypes.c_long),
                ("n", ctypes.c_int * 3), ("ng", ctypes.c_int), ("h", ctypes.c_double * 3),
                ("x0", ctypes.c_double * 3), ("F", ctypes.c_int * 3), ("bc", ctypes.c_int),
                ("has_prev", ctypes.c_int), ("parent", ctypes.c_int), ("obj", ctypes.c_int)]


class OzParams(ctypes.Structure):
    _fields_ = [("kappa1", ctypes.c_double), ("kappa2", ctypes.c_double), ("kappa3", ctypes.c_double),
                ("eta", ctypes.c_double), ("shift_coeff", ctypes.c_double), ("ko_sigma", ctypes.c_double),
                ("w_floor", ctypes.c_double), ("lapse_uses_K", ctypes.c_int)]


def params(kappa1=0.005, kappa2=0.0, kappa3=0.0, eta=0.36, shift_coeff=0.75, ko_sigma=0.5,
           w_floor=1e-10, lapse_uses_K=0) -> OzParams:
    """Defaults: kappa1, kappa2, eta from the paper's run settings (Sec. 3),
    sigma_KO = 0.5 and the 0.75 shift coefficient from Sec. 2.2 / Sec. 2.1.1."""
    return OzParams(kappa1, kappa2, kappa3, eta, shift_coeff, ko_sigma, w_floor, lapse_uses_K)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        geo = [ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
               ctypes.c_double, ctypes.c_double, ctypes.c_double,
               ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.oz_rhs.argtypes = [dp, dp] + geo + [ctypes.POINTER(OzParams), ctypes.c_int]
        L.oz_rhs_points.argtypes = [dp] + geo + [ctypes.POINTER(OzParams), ip, ctypes.c_long, dp, ctypes.c_int]
        L.oz_apply_ghosts.argtypes = [dp, dp, ctypes.c_long] + [ctypes.c_int] * 5
        L.oz_enforce.argtypes = [dp, ctypes.c_long] + [ctypes.c_int] * 5
        L.oz_stage_points.argtypes = [dp, dp, ctypes.c_double] + geo + [ctypes.POINTER(OzParams), ip,
                                                                         ctypes.c_long, dp, ctypes.c_int]
        L.oz_rk4.argtypes = [dp, dp] + geo + [ctypes.POINTER(OzParams), ctypes.c_double, ctypes.c_int,
                                              ctypes.c_int]
        L.oz_constraints.argtypes = [dp, dp, dp] + geo + [ctypes.POINTER(OzParams), ctypes.c_int]
        L.oz_stencil_1d.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        L.oz_bo_advance.argtypes = [ctypes.POINTER(OzLevel), ctypes.c_int, ctypes.POINTER(OzParams), ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int]
        L.oz_prolong.argtypes = [dp, dp, dp, dp, ctypes.c_long, ip, ctypes.c_int, dp, ctypes.c_long, ip, ctypes.c_int,
                                 ip, ctypes.c_int, ctypes.c_int]
        L.oz_restrict.argtypes = [dp, ctypes.c_long, ip, ctypes.c_int, dp, ctypes.c_long, ip, ctypes.c_int, ip,
                                  ctypes.c_int]
        L.oz_transfer_weights.argtypes = [ctypes.c_double, ctypes.c_int, dp, dp, dp, dp]
        L.oz_bo_advance_moving.argtypes = [ctypes.POINTER(OzLevel), ctypes.c_int, ctypes.c_int, dp,
                                           ctypes.POINTER(OzParams), ctypes.c_double, ctypes.c_int, ctypes.c_int]
        L.oz_interp_beta.argtypes = [dp, ctypes.c_long, ip, ctypes.c_int, dp, dp, dp, dp]
        L.oz_regrid.argtypes = [ctypes.POINTER(OzLevel), ctypes.c_int, ctypes.c_int, dp, ctypes.c_int]
        L.oz_exchange.argtypes = [ctypes.POINTER(OzLevel), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oz_mixed_2d.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        for name in ("oz_rhs", "oz_rhs_points", "oz_apply_ghosts", "oz_enforce", "oz_stage_points", "oz_rk4",
                     "oz_stencil_1d", "oz_mixed_2d", "oz_constraints", "oz_bo_advance", "oz_prolong", "oz_restrict",
                     "oz_transfer_weights", "oz_bo_advance_moving", "oz_interp_beta", "oz_regrid", "oz_exchange"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with status {rc}")


def _geo(g):
    """g: dict with n (3), ng, h (3), x0 (3), bc -> ctypes argument tuple (without sf)."""
    n, ng, h, x0 = g["n"], g["ng"], g["h"], g["x0"]
    return (int(n[0]), int(n[1]), int(n[2]), int(ng), float(h[0]), float(h[1]), float(h[2]),
            float(x0[0]), float(x0[1]), float(x0[2]), int(g["bc"]))


def _state(u):
    if u.dtype != np.float64 or not u.flags.c_contiguous or u.ndim != 4 or u.shape[0] != NF:
        raise ValueError("state must be a C-contiguous float64 array of shape (25, Nz, Ny, Nx)")
    return u


def threads_default() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def rhs(u, g, p=None, nthreads=None) -> np.ndarray:
    """Right-hand side on every evolved point (active; plus outer ghosts for a
    Sommerfeld box).  Ghosts of ``u`` must already be valid."""
    _state(u)
    p = p or params()
    out = np.zeros_like(u)
    sf = u[0].size
    _check(lib().oz_rhs(_dp(u), _dp(out), sf, *_geo(g), ctypes.byref(p), nthreads or threads_default()), "rhs")
    return out


def rhs_points(u, g, pts, p=None, nthreads=None) -> np.ndarray:
    """Right-hand side at stored-index points pts (M, 3) as (i, j, k) -> (M, 25)."""
    _state(u)
    p = p or params()
    pts = np.ascontiguousarray(pts, dtype=np.int32)
    out = np.zeros((len(pts), NF))
    _check(lib().oz_rhs_points(_dp(u), u[0].size, *_geo(g), ctypes.byref(p),
                               pts.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(pts), _dp(out),
                               nthreads or threads_default()), "rhs_points")
    return out


def stage_points(u_in, u_n, c_dt, g, pts, p=None, nthreads=None) -> np.ndarray:
    """enforce(u_n + c_dt * rhs(u_in)) at points pts (M, 3) -> (M, 25)."""
    _state(u_in)
    _state(u_n)
    p = p or params()
    pts = np.ascontiguousarray(pts, dtype=np.int32)
    out = np.zeros((len(pts), NF))
    _check(lib().oz_stage_points(_dp(u_in), _dp(u_n), float(c_dt), u_in[0].size, *_geo(g), ctypes.byref(p),
                                 pts.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(pts), _dp(out),
                                 nthreads or threads_default()), "stage_points")
    return out


def apply_ghosts(u, g, shell=None) -> None:
    _state(u)
    n, ng = g["n"], g["ng"]
    sh = None if shell is None else _dp(np.ascontiguousarray(shell, dtype=np.float64))
    _check(lib().oz_apply_ghosts(_dp(u), sh, u[0].size, int(n[0]), int(n[1]), int(n[2]), int(ng), int(g["bc"])),
           "apply_ghosts")


def enforce(u, g) -> None:
    _state(u)
    n, ng = g["n"], g["ng"]
    _check(lib().oz_enforce(_dp(u), u[0].size, int(n[0]), int(n[1]), int(n[2]), int(ng), int(g["bc"])),
           "enforce")


def rk4(u, g, dt, nsteps, p=None, shell=None, nthreads=None) -> None:
    """Advance u in place by nsteps classical RK4 steps of size dt."""
    _state(u)
    p = p or params()
    sh = None
    if shell is not None:
        shell = np.ascontiguousarray(shell, dtype=np.float64)
        sh = _dp(shell)
    _check(lib().oz_rk4(_dp(u), sh, u[0].size, *_geo(g), ctypes.byref(p), float(dt), int(nsteps),
                        nthreads or threads_default()), "rk4")


def constraints(u, g, p=None, nthreads=None):
    """Hamiltonian and momentum constraints (paper Sec. 2.3, vacuum) on the
    active points -> (c (4, Nz, Ny, Nx) with H, M^x, M^y, M^z, L2 norms (4,))."""
    _state(u)
    p = p or params()
    c = np.zeros((4,) + u.shape[1:])
    norms = np.zeros(4)
    _check(lib().oz_constraints(_dp(u), _dp(c), _dp(norms), u[0].size, *_geo(g), ctypes.byref(p),
                                nthreads or threads_default()), "constraints")
    return c, norms


def _ivec(v):
    a = (ctypes.c_int * 3)(*[int(x) for x in v])
    return ctypes.cast(a, ctypes.POINTER(ctypes.c_int)), a


class Level:
    """One patch of a box-in-box hierarchy for bo_advance: its grid, state u
    (advanced in place), the earlier time level `prev` (allocated here), F,
    the parent active cell index of its lower faces (patches >= 1), the
    index of its parent patch (None: the patch listed just before it) and
    the tracked object it follows (-1: a fixed patch)."""

    def __init__(self, grid, u, F=(0, 0, 0), parent=None, obj=-1):
        self.grid = grid
        self.u = _state(u)
        self.prev = np.zeros_like(u)
        self.F = tuple(int(x) for x in F)
        self.has_prev = 0
        self.parent = parent
        self.obj = int(obj)


def _level_array(levels):
    arr = (OzLevel * len(levels))()
    for q, (L, lv) in enumerate(zip(arr, levels)):
        g = lv.grid
        L.u = lv.u.ctypes.data
        L.prev = lv.prev.ctypes.data
        L.sf = lv.u[0].size
        L.n[:] = [int(x) for x in g.n]
        L.ng = int(g.ng)
        L.h[:] = [float(x) for x in g.h]
        L.x0[:] = [float(x) for x in g.x0]
        L.F[:] = list(lv.F)
        L.bc = int(g.bc)
        L.has_prev = lv.has_prev
        L.parent = int(lv.parent) if lv.parent is not None else q - 1
        L.obj = lv.obj
    return arr


def _level_back(arr, levels):
    from dataclasses import replace
    for L, lv in zip(arr, levels):
        lv.has_prev = L.has_prev
        lv.F = tuple(int(x) for x in L.F)
        x0 = tuple(float(x) for x in L.x0)
        if x0 != tuple(float(x) for x in lv.grid.x0):
            lv.grid = replace(lv.grid, x0=x0)


def bo_advance(levels, dt0, nsteps, p=None, nthreads=None) -> None:
    """Berger-Oliger advance of the hierarchy by nsteps root steps of dt0
    (a patch at depth d takes 2^d steps of dt0 / 2^d each)."""
    p = p or params()
    arr = _level_array(levels)
    _check(lib().oz_bo_advance(arr, len(levels), ctypes.byref(p), float(dt0), int(nsteps),
                               nthreads or threads_default()), "bo_advance")
    _level_back(arr, levels)


def _punctures(xp):
    x = np.array(xp, dtype=np.float64)
    single = x.ndim == 1
    x = np.ascontiguousarray(x.reshape(-1, 3))
    return x, single


def bo_advance_moving(levels, xp, dt0, nsteps, p=None, nthreads=None) -> np.ndarray:
    """As bo_advance, with the patches whose obj >= 0 following the
    punctures xp (one row of 3 per object; a single row may be flat),
    each tracked on its object's deepest patch (dx/dt = -beta).  After every
    root step each moving patch shifts by two of its cells toward its
    puncture when its centre is more than two cells away.  Returns the
    final punctures in the shape of xp; grids and F are updated in place."""
    p = p or params()
    x, single = _punctures(xp)
    arr = _level_array(levels)
    _check(lib().oz_bo_advance_moving(arr, len(levels), len(x), _dp(x), ctypes.byref(p), float(dt0),
                                      int(nsteps), nthreads or threads_default()), "bo_advance_moving")
    _level_back(arr, levels)
    return x[0] if single else x


def regrid(levels, xp, nthreads=None) -> None:
    """One regrid of the moving patches toward xp, without a time step."""
    x, _ = _punctures(xp)
    arr = _level_array(levels)
    _check(lib().oz_regrid(arr, len(levels), len(x), _dp(x), nthreads or threads_default()), "regrid")
    _level_back(arr, levels)


def exchange(levels, depth, mode, nthreads=None) -> None:
    """The exchange between the patches at one depth, in place: mode
    "average" (overlapping active cells take their mean) or "ghosts" (ghost
    points inside another patch's active region take its value)."""
    arr = _level_array(levels)
    m = {"average": 0, "ghosts": 1}[mode]
    _check(lib().oz_exchange(arr, len(levels), int(depth), m, nthreads or threads_default()), "exchange")


def interp_beta(u, g, x) -> np.ndarray:
    """4-point Lagrange interpolation of the shift of state u (grid g) at x."""
    _state(u)
    nn, _k1 = _ivec(g.n)
    h = np.ascontiguousarray(g.h, dtype=np.float64)
    x0 = np.ascontiguousarray(g.x0, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    b = np.zeros(3)
    _check(lib().oz_interp_beta(_dp(u), u[0].size, nn, int(g.ng), _dp(h), _dp(x0), _dp(xx), _dp(b)), "interp_beta")
    return b


def prolong(parent_levels, wt, np_, ngp, uc, nc, ngc, F, refl=False, nthreads=None) -> None:
    """Fill every ghost of the child state uc from up to three parent time
    levels (None allowed) combined with the time weights wt; refl: the
    parent's lower z face is a symmetry plane (layers below it read as the
    mirror images, with each field's z parity)."""
    pa = [None if a is None else _dp(_state(a)) for a in parent_levels]
    sfp = next(a for a in parent_levels if a is not None)[0].size
    wt = np.ascontiguousarray(wt, dtype=np.float64)
    pn, _k1 = _ivec(np_)
    cn, _k2 = _ivec(nc)
    fF, _k3 = _ivec(F)
    _check(lib().oz_prolong(pa[0], pa[1], pa[2], _dp(wt), sfp, pn, int(ngp), _dp(_state(uc)), uc[0].size, cn, int(ngc),
                            fF, int(bool(refl)), nthreads or threads_default()), "prolong")


def restrict(uc, nc, ngc, up, np_, ngp, F, nthreads=None) -> None:
    cn, _k1 = _ivec(nc)
    pn, _k2 = _ivec(np_)
    fF, _k3 = _ivec(F)
    _check(lib().oz_restrict(_dp(_state(uc)), uc[0].size, cn, int(ngc), _dp(_state(up)), up[0].size, pn, int(ngp), fF,
                             nthreads or threads_default()), "restrict")


def transfer_weights(theta, quadratic):
    """(time weights (3,), prolongation weights for even / odd child cells
    (6,) each, restriction weights (4,))."""
    out = [np.zeros(3), np.zeros(6), np.zeros(6), np.zeros(4)]
    _check(lib().oz_transfer_weights(float(theta), int(quadratic), *[_dp(o) for o in out]), "transfer_weights")
    return tuple(out)


def stencil_1d(op, f, h, beta_sign=1.0) -> np.ndarray:
    """op: 'd1', 'd2', 'up', 'ko' applied at interior points [3, n-3)."""
    code = {"d1": 0, "d2": 1, "up": 2, "ko": 3}[op]
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    _check(lib().oz_stencil_1d(code, _dp(f), len(f), float(h), float(beta_sign), _dp(out)), "stencil_1d")
    return out


def mixed_2d(f, hx, hy) -> np.ndarray:
    """D1_x(D1_y f) on a (ny, nx) array at interior points."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    _check(lib().oz_mixed_2d(_dp(f), f.shape[1], f.shape[0], float(hx), float(hy), _dp(out)), "mixed_2d")
    return out
