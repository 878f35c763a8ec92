"""Seeded synthetic inputs for the Z4c evolution step.

This module builds initial data and box geometry only.  It holds none of the
method's arithmetic (no stencil, right-hand side, RK4, ghost fill or
constraint enforcement); both the HIP path and the test oracle consume the
arrays it returns.

Grids are cell-centred (paper Sec. 2.2.1: cell-centred staggering): the centre
of stored point i is x0 + (i - ng) h, active cells are i in [ng, ng + n).
Arrays are float64 with shape (25, Nz, Ny, Nx), x fastest.

Field order (25 evolved fields of paper Sec. 2.1.1 plus Theta of the Z4c
prescription):

    0 W | 1-6 gt_xx gt_xy gt_xz gt_yy gt_yz gt_zz | 7 Khat
    8-13 At_xx .. At_zz | 14-16 Gt^x Gt^y Gt^z | 17 Theta | 18 alpha
    19-21 beta^x..z | 22-24 B^x..z
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

NF = 25
NG = 3
BC_PERIODIC, BC_SOMMERFELD, BC_COPY, BC_EQUATORIAL = 0, 1, 2, 3

FIELD_NAMES = ["W", "gt_xx", "gt_xy", "gt_xz", "gt_yy", "gt_yz", "gt_zz", "Khat",
               "At_xx", "At_xy", "At_xz", "At_yy", "At_yz", "At_zz", "Gt_x", "Gt_y", "Gt_z",
               "Theta", "alpha", "beta_x", "beta_y", "beta_z", "B_x", "B_y", "B_z"]

# value of each field in flat space (W = alpha = 1, gt = identity, the rest 0)
FLAT = np.array([1, 1, 0, 0, 1, 0, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 0], dtype=np.float64)

# sign of each field under the pi rotation (x, y, z) -> (-x, -y, z) (paper Sec. 3.2):
# scalars +, vector x/y components -, tensor xz/yz components -
PI_PARITY = np.array([+1, +1, +1, -1, +1, -1, +1, +1, +1, +1, -1, +1, -1, +1, -1, -1, +1,
                      +1, +1, -1, -1, +1, -1, -1, +1], dtype=np.float64)


# sign of each field under the reflection z -> -z: (-1)^(number of z indices)
Z_PARITY = np.array([+1, +1, +1, -1, +1, -1, +1, +1, +1, +1, -1, +1, -1, +1, +1, +1, -1,
                     +1, +1, +1, +1, -1, +1, +1, -1], dtype=np.float64)


@dataclass
class Grid:
    """One box: active cells n, ghost width ng, spacing h, centre of the first
    active cell x0, boundary kind bc."""
    n: tuple
    h: tuple
    x0: tuple
    bc: int
    ng: int = NG

    @property
    def shape(self):
        return (NF,) + tuple(int(self.n[d]) + 2 * self.ng for d in (2, 1, 0))

    @property
    def stored(self) -> int:
        s = self.shape
        return s[1] * s[2] * s[3]

    @property
    def active(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def as_dict(self) -> dict:
        return {"n": tuple(int(v) for v in self.n), "ng": int(self.ng), "h": tuple(float(v) for v in self.h),
                "x0": tuple(float(v) for v in self.x0), "bc": int(self.bc)}

    def coords(self):
        """Cell-centre coordinates of every stored point, each (Nz, Ny, Nx)."""
        ax = [self.x0[d] + (np.arange(int(self.n[d]) + 2 * self.ng) - self.ng) * self.h[d] for d in range(3)]
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        return X, Y, Z

    def active_mask(self):
        m = np.zeros(self.shape[1:], dtype=bool)
        g = self.ng
        m[g:g + self.n[2], g:g + self.n[1], g:g + self.n[0]] = True
        return m


def centered_grid(n, h, center=(0.0, 0.0, 0.0), bc=BC_PERIODIC, ng=NG) -> Grid:
    """Cubic-cell box of n cells per side (int or 3-tuple) centred on `center`."""
    if np.isscalar(n):
        n = (int(n),) * 3
    if np.isscalar(h):
        h = (float(h),) * 3
    x0 = tuple(center[d] - 0.5 * (n[d] - 1) * h[d] for d in range(3))
    return Grid(tuple(int(v) for v in n), tuple(float(v) for v in h), x0, bc, ng)


def flat_state(g: Grid) -> np.ndarray:
    u = np.zeros(g.shape)
    u[:] = FLAT[:, None, None, None]
    return u


def plane_wave_state(g: Grid, amp=1e-6, wavelength=3.2, noise=1e-10, seed=1) -> np.ndarray:
    """Linearised '+'-polarised gravitational wave travelling along +z in TT
    gauge (alpha = 1, beta = 0): gamma_xx = 1 + hw, gamma_yy = 1 - hw,
    hw = amp sin(2 pi z / L), K_xx = -K_yy = hw'/2.  Conformal variables from
    their definitions (paper Sec. 2.1.1).  Optional seeded uniform noise of
    size `noise` is added to every field on the active points only."""
    _, _, Z = g.coords()
    k = 2.0 * np.pi / wavelength
    hw = amp * np.sin(k * Z)
    dhw = amp * k * np.cos(k * Z)
    gxx, gyy = 1.0 + hw, 1.0 - hw
    det = gxx * gyy
    W = det ** (-1.0 / 6.0)
    Kxx, Kyy = 0.5 * dhw, -0.5 * dhw
    K = Kxx / gxx + Kyy / gyy
    u = flat_state(g)
    u[0] = W
    u[1] = W * W * gxx
    u[4] = W * W * gyy
    u[6] = W * W
    u[7] = K
    u[8] = W * W * (Kxx - gxx * K / 3.0)
    u[11] = W * W * (Kyy - gyy * K / 3.0)
    u[13] = W * W * (-K / 3.0)
    # Gt^z = -d_z gt^zz with gt^zz = W^-2 = det^(1/3)
    u[16] = -(1.0 / 3.0) * det ** (-2.0 / 3.0) * (-2.0 * hw * dhw)
    if noise:
        n = g.n
        rng = np.random.default_rng(seed)
        eps = rng.uniform(-noise, noise, (NF, n[2], n[1], n[0]))
        s = g.ng
        u[:, s:s + n[2], s:s + n[1], s:s + n[0]] += eps
    return u


def brill_lindquist_psi(X, Y, Z, masses=(0.5, 0.5), centres=((5.0, 0.0, 0.0), (-5.0, 0.0, 0.0))):
    """Conformal factor psi = 1 + sum m_a / (2 r_a); the two terms are summed
    before adding 1 so that the result is exactly symmetric under x -> -x."""
    terms = [m / (2.0 * np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)) for m, c in zip(masses, centres)]
    s = terms[0]
    for t in terms[1:]:
        s = s + t
    return 1.0 + s


def brill_lindquist_state(g: Grid, masses=(0.5, 0.5), centres=((5.0, 0.0, 0.0), (-5.0, 0.0, 0.0))) -> np.ndarray:
    """Time-symmetric two-puncture data: gamma = psi^4 delta, K_ij = 0, so
    W = psi^-2, gt = delta, and a pre-collapsed lapse alpha = W."""
    X, Y, Z = g.coords()
    psi = brill_lindquist_psi(X, Y, Z, masses, centres)
    u = flat_state(g)
    u[0] = psi ** -2.0
    u[18] = u[0]
    return u


def pi_symmetrize(u: np.ndarray) -> np.ndarray:
    """Replace every value with x < 0 by the parity-signed value at its
    partner (-x, -y, z) (paper Sec. 3.2).  Boxes must be symmetric about the
    z axis so that stored index i maps to Nx-1-i and j to Ny-1-j."""
    out = u.copy()
    Nx = u.shape[3]
    half = Nx // 2
    mirrored = u[:, :, ::-1, ::-1] * PI_PARITY[:, None, None, None]
    out[:, :, :, :half] = mirrored[:, :, :, :half]
    return out


def random_strong_field_state(g: Grid, seed=7, amp=0.1, kmax=3) -> np.ndarray:
    """Every field = flat value + amp * smooth random Fourier sum (periodic in
    the active box, wavenumbers <= kmax).  Diagonal metric components stay
    near 1 and off-diagonals near 0, so gt is positive definite and W, alpha
    stay inside [0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    X, Y, Z = g.coords()
    L = [g.n[d] * g.h[d] for d in range(3)]
    u = flat_state(g)
    for f in range(NF):
        acc = np.zeros_like(X)
        for _ in range(4):
            kx, ky, kz = rng.integers(-kmax, kmax + 1, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            a = rng.uniform(-1, 1)
            acc += a * np.cos(2 * np.pi * (kx * X / L[0] + ky * Y / L[1] + kz * Z / L[2]) + ph)
        u[f] += amp * acc / 4.0
    return u


def shell_of(u: np.ndarray, g: Grid) -> np.ndarray:
    """Ghost values of u in the canonical shell order: stored points that are
    not active, visited with k outermost and i fastest.  Shape (25, nshell)."""
    m = ~g.active_mask()
    return np.ascontiguousarray(u[:, m])


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def config_plane_wave(n=32):
    """32^3 periodic box, h = 0.1 ([-1.6, 1.6]^3), plane wave amplitude 1e-6
    plus uniform noise +-1e-10 (seed 1); one RK4 step of dt = 0.5 h."""
    g = centered_grid(n, 3.2 / n, bc=BC_PERIODIC)
    return g, plane_wave_state(g), 0.5 * g.h[0]


def config_punctures(n=128, extent=32.0):
    """n^3 Sommerfeld box over [-16, 16]^3 with two Brill-Lindquist punctures
    (m = 0.5 each at x = +-5, separation 10), lapse alpha = W, pi-symmetrised.
    dt = 0.5 h (Courant factor 0.5, paper Sec. 2.2)."""
    g = centered_grid(n, extent / n, bc=BC_SOMMERFELD)
    return g, pi_symmetrize(brill_lindquist_state(g)), 0.5 * g.h[0]


def z_symmetrize(u: np.ndarray) -> np.ndarray:
    """Make a box that is symmetric about z = 0 (stored index k <-> Nz-1-k)
    exactly reflection-symmetric: the average of u and its parity-signed
    mirror image."""
    return 0.5 * (u + u[:, ::-1, :, :] * Z_PARITY[:, None, None, None])


def upper_half(u: np.ndarray, ng: int = NG) -> np.ndarray:
    """Stored points of the z >= 0 half of a z-symmetric box (an even number
    of active layers) together with ng layers below the plane."""
    nz = u.shape[1] - 2 * ng
    return np.ascontiguousarray(u[:, nz // 2:, :, :])


def config_punctures_equatorial(n=128, extent=32.0):
    """The z >= 0 half (n x n x n/2 cells) of the n^3 two-puncture box, with
    equatorial reflection symmetry at z = 0 and Sommerfeld outer faces: the
    same physical problem for half the cells (paper Sec. 2.4)."""
    h = extent / n
    g = Grid((n, n, n // 2), (h, h, h), (-0.5 * (n - 1) * h, -0.5 * (n - 1) * h, 0.5 * h), BC_EQUATORIAL)
    return g, pi_symmetrize(brill_lindquist_state(g)), 0.5 * h


HIERARCHY_SIZES = (160, 144, 128, 112, 96, 96, 80, 72, 64)


@dataclass
class Box:
    grid: Grid
    state: np.ndarray
    shell: np.ndarray
    dt: float
    level: int = 0


def config_hierarchy(sizes=HIERARCHY_SIZES, h0=2.0, noise=1e-10):
    """Box-in-box stand-in of 9 levels (ratio 2) with uneven box sizes:
    level l has sizes[l]^3 cells at h = h0 / 2^l; levels 0-4 are centred on
    the origin, levels 5-8 on the puncture at (+5, 0, 0) (the moving-level
    patch of paper Sec. 2.2.1).  Brill-Lindquist data everywhere.  Ghost
    shells are the analytic data at the ghost points plus seeded uniform
    noise (seed 100 + l), fixed in time; each box uses dt = 0.5 h."""
    boxes = []
    for lev, n in enumerate(sizes):
        h = h0 / 2 ** lev
        centre = (0.0, 0.0, 0.0) if lev <= 4 else (5.0, 0.0, 0.0)
        g = centered_grid(n, h, center=centre, bc=BC_COPY)
        u = brill_lindquist_state(g)
        sh = shell_of(u, g)
        if noise:
            sh = sh + np.random.default_rng(100 + lev).uniform(-noise, noise, sh.shape)
        boxes.append(Box(g, u, np.ascontiguousarray(sh), 0.5 * h, lev))
    return boxes


def bo_level_grids(nlev=6, n=64, h0=4.0, bc0=BC_SOMMERFELD, ng=NG):
    """Fixed levels of a box-in-box hierarchy for Berger-Oliger subcycling
    (paper Sec. 2.2.1): level l is an n^3 box centred on the origin with
    h = h0 / 2^l, so each child covers the central half of its parent; its
    lower faces sit on parent cell F = n/4.  Returns [(grid, F)]."""
    out = []
    for lev in range(nlev):
        h = h0 / 2 ** lev
        g = centered_grid(n, h, bc=bc0 if lev == 0 else BC_COPY, ng=ng)
        out.append((g, (0, 0, 0) if lev == 0 else (n // 4,) * 3))
    return out


def child_grid(gp: Grid, n, center, ng=NG):
    """A patch of n cells per side (int or 3-tuple) refining gp 2:1, centred
    on `center`, with its lower faces on parent cell faces.  Returns (grid,
    F), F the parent active cell index of the lower faces."""
    if np.isscalar(n):
        n = (int(n),) * 3
    hc = tuple(0.5 * float(h) for h in gp.h)
    F, x0 = [], []
    for d in range(3):
        face = (center[d] - 0.5 * n[d] * hc[d] - (gp.x0[d] - 0.5 * gp.h[d])) / gp.h[d]
        f = int(round(face))
        if abs(face - f) > 1e-9:
            raise ValueError("the patch's faces do not fall on parent cell faces")
        F.append(f)
        x0.append(gp.x0[d] + (f - 0.25) * gp.h[d])
    return Grid(tuple(int(v) for v in n), hc, tuple(x0), BC_COPY, ng), tuple(F)


def pair_hierarchy(root_n, h0, centers, moving, fixed=(), bc0=BC_PERIODIC, ng=NG):
    """Patches of a hierarchy with moving levels (paper Sec. 2.2.1, Fig. 1):
    a root of root_n^3 cells centred on the origin, fixed levels of sizes
    `fixed` centred on the origin, then moving levels of sizes `moving`,
    each with one patch per object centred on centers[o].  Returns
    [(grid, F, parent, obj)] with parents listed before their children and
    the patches of one depth in object order."""
    out = [(centered_grid(root_n, h0, bc=bc0, ng=ng), (0, 0, 0), -1, -1)]
    for n in fixed:
        g, F = child_grid(out[-1][0], n, (0.0, 0.0, 0.0), ng)
        out.append((g, F, len(out) - 1, -1))
    last = {o: len(out) - 1 for o in range(len(centers))}
    for n in moving:
        for o, c in enumerate(centers):
            g, F = child_grid(out[last[o]][0], n, c, ng)
            out.append((g, F, last[o], o))
            last[o] = len(out) - 1
    return out


def upper_half_patches(patches, states):
    """The upper half (z > 0) of a hierarchy whose patches are all centred on
    z = 0 with z-symmetric data: the root becomes an equatorial box, every
    other patch a patch whose lower z face is the symmetry plane (F_z = 0)."""
    out_p, out_s = [], []
    for (g, F, par, obj), u in zip(patches, states):
        if g.n[2] % 2 or abs(g.x0[2] + 0.5 * (g.n[2] - 1) * g.h[2]) > 1e-12 * g.h[2]:
            raise ValueError("every patch must be centred on z = 0 with an even z extent")
        gh = Grid((g.n[0], g.n[1], g.n[2] // 2), g.h, (g.x0[0], g.x0[1], 0.5 * g.h[2]),
                  BC_EQUATORIAL if par < 0 else g.bc, g.ng)
        out_p.append((gh, (F[0], F[1], 0) if par >= 0 else tuple(F), par, obj))
        out_s.append(upper_half(u, g.ng))
    return out_p, out_s


def config_bbh_moving(root_n=128, h0=2.0, fixed=(128, 128, 128), moving=(64, 64, 64), sep=10.0, equatorial=False,
                      lag=0.0):
    """The binary-black-hole layout of Sec. 2.2.1 (Fig. 1): a Sommerfeld
    root of root_n^3 cells (spacing h0) and fixed levels centred on the
    origin, then moving levels with one patch per puncture, centred on
    x = +-sep/2, on two Brill-Lindquist punctures (m = 0.5 each), alpha = W.
    The punctures sit at x = +-(sep/2 - lag): lag > 0 puts them that far
    inside their patches' centres, as between two regrids of a running
    evolution.  equatorial: only the upper half (z > 0), every patch on the
    symmetry plane.  Returns (patches [(grid, F, parent, obj)], states, root
    step dt0 = 0.5 h0, puncture positions (2, 3))."""
    centers = [(-0.5 * sep, 0.0, 0.0), (0.5 * sep, 0.0, 0.0)]
    a = 0.5 * sep - lag
    punct = ((a, 0.0, 0.0), (-a, 0.0, 0.0))  # the +x puncture first: the pair's sum is mirror-safe
    pt = pair_hierarchy(root_n, h0, centers, moving, fixed, bc0=BC_SOMMERFELD)
    states = [brill_lindquist_state(g, centres=punct) for g, *_ in pt]
    if equatorial:
        pt, states = upper_half_patches(pt, [z_symmetrize(u) for u in states])
    return pt, states, 0.5 * h0, np.array([(-a, 0.0, 0.0), (a, 0.0, 0.0)])


def config_bo_hierarchy(nlev=6, n=64, h0=4.0):
    """Two-puncture Brill-Lindquist data on every level of bo_level_grids,
    pi-symmetrised; coarse step dt0 = 0.5 h0 (level l: 0.5 h0 / 2^l)."""
    levels = [(g, pi_symmetrize(brill_lindquist_state(g)), F) for g, F in bo_level_grids(nlev, n, h0)]
    return levels, 0.5 * h0
