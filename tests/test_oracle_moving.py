"""Pins of the oracle's moving levels (paper Sec. 2.2.1): puncture tracking
dx/dt = -beta on the finest level and two-cell patch shifts with the newly
covered cells prolonged from the parent.

* The beta interpolation reproduces cubics (4-point Lagrange per direction)
  and misses quartics.
* A regrid moves a patch by two of its cells: cells it already covered keep
  their values bit for bit, new ones hold the parent's degree-5 polynomial
  exactly (6th-order prolongation), and F and x0 move by one parent cell.
* A pure gauge translation (flat metric, constant shift, B = 0, eta = 0:
  beta is constant and nothing else moves) is tracked exactly,
  x(t) = x0 - beta t, the patches follow the shift decisions replayed here
  from that trajectory, and the state stays constant through every shift
  (to rounding: prolonged cells carry the rounding of the weights' sum).
"""
import numpy as np
import pytest

from paper_2607_08743_amd import inputs as I

NG = 3


def _poly(X, Y, Z, deg):
    return (1 + 0.1 * X) ** deg * (1 - 0.07 * Y) ** deg * (1 + 0.05 * Z) ** deg + 0.3 * X - 0.2 * Y * Z


def test_interp_beta_cubic(oz):
    g = I.centered_grid((16, 14, 12), (0.5, 0.4, 0.3), bc=I.BC_COPY)
    X, Y, Z = g.coords()
    rng = np.random.default_rng(2)
    for deg, exact in ((3, True), (4, False)):
        u = I.flat_state(g)
        for a in range(3):
            u[19 + a] = _poly(X, Y, Z, deg) * (a + 1)
        errs = []
        for _ in range(20):
            x = rng.uniform(-2.0, 2.0, 3) * np.array([1.0, 1.0, 0.6])  # stencils on active cells
            b = oz.interp_beta(u, g, x)
            want = _poly(*x, deg) * np.arange(1, 4)
            errs.append(np.abs(b - want).max() / np.abs(want).max())
        if exact:
            assert max(errs) < 1e-13, max(errs)
        else:
            assert max(errs) > 1e-9, max(errs)


def test_regrid_shift_and_prolong(oz):
    grids = I.bo_level_grids(3, 24, 1.0)
    lv = []
    for g, F in grids:
        X, Y, Z = g.coords()
        u = I.flat_state(g)
        for f in range(25):
            u[f] = _poly(X, Y, Z, 5) + f
        lv.append(oz.Level(g, u, F, obj=0 if lv else -1))
    old = [(L.u.copy(), L.grid, L.F) for L in lv]
    h2 = lv[2].grid.h[0]
    xp = np.array([3.0 * h2, -2.6 * h2, 0.4 * h2])  # past the threshold in x (+) and y (-)
    oz.regrid(lv, xp)
    # level 1 (h = 0.5): the puncture is within 2 of its cells: unchanged
    assert np.array_equal(lv[1].u, old[1][0]) and lv[1].F == old[1][2]
    # level 2 shifts by (+1, -1, 0) parent cells
    L = lv[2]
    assert L.F == (old[2][2][0] + 1, old[2][2][1] - 1, old[2][2][2])
    assert np.allclose(np.array(L.grid.x0) - np.array(old[2][1].x0), [2 * h2, -2 * h2, 0.0], rtol=0, atol=1e-15)
    X, Y, Z = L.grid.coords()
    m = L.grid.active_mask()
    for f in (0, 7, 19):
        want = _poly(X, Y, Z, 5) + f
        err = np.abs(L.u[f][m] - want[m]).max() / np.abs(want[m]).max()
        assert err < 1e-13, (f, err)
    # cells covered before and after keep their values exactly
    ng, n = NG, 24
    new_act = L.u[:, ng:ng + n, ng:ng + n, ng:ng + n]
    old_act = old[2][0][:, ng:ng + n, ng:ng + n, ng:ng + n]
    assert np.array_equal(new_act[:, :, 2:, :n - 2], old_act[:, :, :n - 2, 2:])


def test_gauge_translation_tracked_exactly(oz):
    beta = np.array([0.3, -0.2, 0.1])
    grids = I.bo_level_grids(3, 24, 1.0, bc0=I.BC_PERIODIC)
    lv = []
    for g, F in grids:
        u = I.flat_state(g)
        u[19:22] = beta[:, None, None, None]
        lv.append(oz.Level(g, u, F, obj=0 if lv else -1))
    p = oz.params(eta=0.0)
    dt0 = 0.5
    xp = np.array([0.05, -0.1, 0.02])
    x = xp.copy()
    # expected patch centres, replayed from the exact trajectory
    cen = {l: np.array([lv[l].grid.x0[d] + 0.5 * (lv[l].grid.n[d] - 1) * lv[l].grid.h[d] for d in range(3)])
           for l in (1, 2)}
    nshift = 0
    for step in range(1, 9):
        x = oz.bo_advance_moving(lv, x, dt0, 1, p)
        exact = xp - beta * step * dt0
        assert np.abs(x - exact).max() < 1e-14, (step, x, exact)
        for l in (1, 2):
            h = lv[l].grid.h[0]
            d = exact - cen[l]
            sh = np.where(d > 2 * h, 1, np.where(d < -2 * h, -1, 0))
            cen[l] = cen[l] + 2 * h * sh
            nshift += int(np.abs(sh).sum())
            got = np.array([lv[l].grid.x0[i] + 0.5 * (lv[l].grid.n[i] - 1) * lv[l].grid.h[i] for i in range(3)])
            assert np.allclose(got, cen[l], rtol=0, atol=1e-14), (step, l)
        for L in lv:
            m = L.grid.active_mask()
            want = I.flat_state(L.grid)
            want[19:22] = beta[:, None, None, None]
            # prolonged cells carry the rounding of the weights' sum (a few
            # ulp), which the stencils then amplify by 1/h^2 step after step
            assert np.abs(L.u[:, m] - want[:, m]).max() < 1e-12
    assert nshift >= 2  # the patches did move
