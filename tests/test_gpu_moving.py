"""GPU moving levels (z4c_hier_set_moving): puncture tracking on the finest
level and two-cell patch shifts, against the oracle's moving hierarchy, and
the exact pure-gauge translation (flat metric, constant shift, B = 0,
eta = 0) in which the puncture moves at -beta and the state stays constant
through every shift."""
import numpy as np
import pytest

from gpu_helpers import normrel, to_host
from paper_2607_08743_amd import inputs as I
from paper_2607_08743_amd import z4c

pytestmark = pytest.mark.gpu
TOL = 1e-12


def test_moving_gauge_translation_exact():
    print("case: moving levels, pure gauge translation", flush=True)
    beta = np.array([0.3, -0.2, 0.1])
    levels = []
    for l, (g, F) in enumerate(I.bo_level_grids(3, 24, 1.0, bc0=I.BC_PERIODIC)):
        u = I.flat_state(g)
        u[19:22] = beta[:, None, None, None]
        levels.append((g, u, F, l - 1, 0 if l else -1))
    dt0 = 0.5
    xp = np.array([0.05, -0.1, 0.02])
    H = z4c.Hierarchy(levels, dt0, params=z4c.default_params(eta=0.0))
    H.set_moving(xp)
    x0_start = [tuple(lv[0].x0) for lv in levels]
    for step in range(1, 9):
        H.advance(1, use_graph=True)
        x, F, x0 = H.puncture()
        exact = xp - beta * step * dt0
        assert np.abs(x[0] - exact).max() < 1e-14, (step, x, exact)
    assert x0[2] != x0_start[2]  # the finest patch moved
    for (g, *_), u, xl in zip(levels, H.u, x0):
        gg = I.Grid(g.n, g.h, xl, g.bc, g.ng)
        m = gg.active_mask()
        want = I.flat_state(gg)
        want[19:22] = beta[:, None, None, None]
        assert np.abs(to_host(u)[:, m] - want[:, m]).max() < 1e-12
    H.close()


def _moving_levels(beta, seed=12):
    out = []
    for l, (g, F) in enumerate(I.bo_level_grids(3, 24, 1.0)):
        u = I.brill_lindquist_state(g)
        u = u + 1e-3 * (I.random_strong_field_state(g, seed=seed) - I.flat_state(g))
        u[19:22] += beta[:, None, None, None]
        out.append((g, u, F, l - 1, 0 if l else -1))
    return out


def _oracle_moving(oz, levels, xp, dt0, nsteps, perturb=None):
    lv = []
    for l, (g, u, F, *_) in enumerate(levels):
        v = u.copy()
        if perturb is not None:
            v = v + np.spacing(v) * perturb.choice([-1.0, 1.0], size=v.shape)
        lv.append(oz.Level(g, v, F, obj=0 if l >= 1 else -1))
    x = oz.bo_advance_moving(lv, xp, dt0, nsteps)
    return lv, x


def test_moving_parity_with_oracle(oz):
    """Brill-Lindquist data plus a smooth perturbation and a constant shift
    that carries the tracked point across the finest level's shift
    threshold: puncture position, patch placement and every level's state
    against the oracle after 4 coarse steps."""
    print("case: moving levels vs oracle, 3 levels of 24^3, 4 coarse steps", flush=True)
    beta = np.array([0.35, 0.0, -0.15])
    levels = _moving_levels(beta)
    dt0 = 0.5
    xp = np.array([0.1, 0.05, -0.05])
    H = z4c.Hierarchy(levels, dt0)
    H.set_moving(xp)
    H.advance(4, use_graph=True)
    x, F, x0 = H.puncture()
    got = [to_host(u) for u in H.u]
    H.close()
    lv, xr = _oracle_moving(oz, levels, xp, dt0, 4)
    alt, _ = _oracle_moving(oz, levels, xp, dt0, 4, perturb=np.random.default_rng(0))
    print("puncture gpu", x, "oracle", xr)
    assert np.abs(x[0] - xr).max() <= 1e-12
    assert x0[2] != tuple(levels[2][0].x0)  # the finest patch moved
    for l, L in enumerate(lv):
        assert F[l] == L.F and np.allclose(x0[l], L.grid.x0, rtol=0, atol=1e-14), l
        m = L.grid.active_mask()
        if l == 0:
            m = np.ones_like(m)  # Sommerfeld ghosts are evolved too
        e = normrel(got[l], L.u, m)
        sens = normrel(alt[l].u, L.u, m)
        print(f"level {l} normrel:", " ".join(f"{v:.1e}" for v in e))
        print(f"level {l} oracle 1-ulp sensitivity:", " ".join(f"{v:.1e}" for v in sens))
        assert np.all(e <= np.maximum(TOL, 20 * sens)), (l, e)
        assert np.abs(got[l][:, m] - L.u[:, m]).max() <= TOL * np.abs(L.u[:, m]).max()


def _edge_levels(F1, xp_off):
    """Root 32^3 (h = 1, periodic) and one moving 24^3 child (h = 1/2) whose
    lower faces sit on root cell F1; flat data with a small constant shift."""
    root = I.centered_grid(32, 1.0, bc=I.BC_PERIODIC)
    F = (F1, 10, 10)
    x0 = tuple(root.x0[d] + (F[d] - 0.25) * root.h[d] for d in range(3))
    child = I.Grid((24, 24, 24), (0.5,) * 3, x0, I.BC_COPY, 3)
    lv = []
    for g, Fl, par, obj in ((root, (0, 0, 0), -1, -1), (child, F, 0, 0)):
        u = I.flat_state(g)
        u[19] = 0.01
        lv.append((g, u, Fl, par, obj))
    centre = np.array([x0[d] + 0.5 * 23 * 0.5 for d in range(3)])
    return lv, centre + np.asarray(xp_off)


def test_moving_shift_out_of_parent_is_an_error():
    """A patch already at the last root cell its stencils allow (F = 16 for a
    24^3 child of a 32^3 root: its last ghost, child cell 26, reads root cells
    up to F + 15) with its puncture three of its cells ahead: the regrid after
    the first root step refuses the shift, as the oracle's does."""
    print("case: moving patch shift out of its parent", flush=True)
    lv, xp = _edge_levels(16, (1.5, 0.0, 0.0))
    H = z4c.Hierarchy(lv, 0.5, params=z4c.default_params(eta=0.0))
    H.set_moving(xp)
    with pytest.raises(z4c.Z4cError, match="prolongation stencil leaves"):
        H.advance(1)
    H.close()


def test_puncture_outside_active_cells_is_an_error():
    """A puncture whose 4-point stencil would need a ghost of its patch: the
    tracking kernel flags it and the advance reports it."""
    print("case: puncture stencil outside the active cells", flush=True)
    lv, xp = _edge_levels(10, (-5.8, 0.0, 0.0))  # 0.2 of a cell inside the first active cell
    H = z4c.Hierarchy(lv, 0.5, params=z4c.default_params(eta=0.0))
    H.set_moving(xp)
    with pytest.raises(z4c.Z4cError, match="left the active cells"):
        H.advance(1)
    H.close()


def test_failed_regrid_keeps_moved_patches_consistent():
    """Two moving 24^3 patches of a 32^3 root; patch 2 already at the last
    root cell its stencils allow.  Both punctures drift +x (constant shift)
    and cross the shift threshold in the regrid after the second root step:
    patch 1 moves, then patch 2's move is refused.  Patch 1 has moved all the
    same, so the next step must use its new position: that step (which fails
    the same way in its regrid) gives bitwise the same states from the
    captured-graph path (whose graph, captured at the second step, holds
    patch 1's old position and must be rebuilt) as from direct launches."""
    print("case: regrid error after another patch moved, graph vs direct", flush=True)
    root = I.centered_grid(32, 1.0, bc=I.BC_PERIODIC)
    lv, xp = [], []
    for q, F in enumerate(((0, 0, 0), (4, 10, 10), (16, 10, 10))):
        g = root
        if q:
            x0 = tuple(root.x0[d] + (F[d] - 0.25) * root.h[d] for d in range(3))
            g = I.Grid((24, 24, 24), (0.5,) * 3, x0, I.BC_COPY, 3)
            xp.append([x0[d] + 0.5 * 23 * 0.5 + (0.85 if d == 0 else 0.0) for d in range(3)])
        u = I.flat_state(g) + 1e-3 * (I.random_strong_field_state(g, seed=80 + q) - I.flat_state(g))
        u[19] -= 0.2  # beta^x = -0.2: the punctures move by +0.1 per root step
        lv.append((g, u, F, 0 if q else -1, q - 1))
    xp = np.array(xp)
    out = []
    for use_graph in (True, False):
        H = z4c.Hierarchy(lv, 0.5)
        H.set_moving(xp)
        H.advance(1, use_graph=use_graph)
        assert H.puncture()[1][1:] == [(4, 10, 10), (16, 10, 10)]  # under the threshold
        with pytest.raises(z4c.Z4cError, match="regrid of patch 2"):
            H.advance(1, use_graph=use_graph)
        assert H.puncture()[1][1:] == [(5, 10, 10), (16, 10, 10)]
        with pytest.raises(z4c.Z4cError, match="regrid of patch 2"):
            H.advance(1, use_graph=use_graph)
        out.append(([to_host(u) for u in H.u], H.puncture()))
        H.close()
    (a, (xa, Fa, _)), (b, (xb, Fb, _)) = out
    assert Fa == Fb and np.array_equal(xa, xb)
    for q in range(3):
        assert np.array_equal(a[q], b[q]), q
