"""Pins of the oracle's box-in-box Berger-Oliger hierarchy (paper Sec.
2.2.1): the transfer operators against exact polynomial reproduction and
the textbook weight values, and the subcycled driver against exact
solutions and its own invariants.

* Prolongation (6th-order Lagrange, 2:1 cell-centred): reproduces every
  polynomial of degree <= 5 in each variable at the child ghost centres,
  and fails to reproduce degree 6 (so the stencil is not wider than
  claimed).  Weights checked against an exact rational solve of the moment
  equations.
* Restriction (4th-order Lagrange): weights (-1, 9, 9, -1)/16; reproduces
  cubics.
* Time interpolation: quadratic through (t_{n-1}, t_n, t_{n+1}), linear
  through (t_n, t_{n+1}) without an earlier level.
* Driver: flat space stays exactly flat; a constant shift driven by a
  constant B with eta = 0 (beta = beta0 + 0.75 B t exactly, everything else
  flat) is reproduced on every level after one coarse step, which needs the
  right number of substeps per level and the right time for every ghost
  fill; after a step the parent's covered cells equal the restriction of
  the child.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_2607_08743_amd import inputs as I

NG = 3


def _solve_moments(nodes, x):
    """Exact rational Lagrange weights: sum_m w_m nodes_m^k = x^k, k < len."""
    n = len(nodes)
    A = [[Fraction(nd) ** k for nd in nodes] for k in range(n)]
    b = [Fraction(x) ** k for k in range(n)]
    for c in range(n):  # Gauss-Jordan
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        b[c], b[piv] = b[piv], b[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [a - f * p for a, p in zip(A[r], A[c])]
                b[r] -= f * b[c]
    return [b[i] / A[i][i] for i in range(n)]


def test_transfer_weights(oz):
    wt, pe, po, r = oz.transfer_weights(0.25, 1)
    ref_even = _solve_moments([-3, -2, -1, 0, 1, 2], Fraction(-1, 4))
    ref_odd = _solve_moments([-2, -1, 0, 1, 2, 3], Fraction(1, 4))
    assert np.allclose(pe, [float(v) for v in ref_even], rtol=0, atol=1e-16)
    assert np.allclose(po, [float(v) for v in ref_odd], rtol=0, atol=1e-16)
    assert np.array_equal(r, np.array([-1.0, 9.0, 9.0, -1.0]) / 16.0)
    for theta in (0.0, 0.25, 0.5, 0.75, 1.0):
        wq, *_ = oz.transfer_weights(theta, 1)
        for k in range(3):  # quadratic in time, nodes -1, 0, 1
            assert abs(wq[0] * (-1.0) ** k + wq[1] * (0.0 ** k) + wq[2] * 1.0 - theta ** k) < 1e-15
        wl, *_ = oz.transfer_weights(theta, 0)
        assert wl[0] == 0.0 and abs(wl[1] - (1 - theta)) < 1e-16 and abs(wl[2] - theta) < 1e-16


def _parent_child(np_=(24, 22, 20), nc=(16, 12, 8), F=(4, 5, 6)):
    """Parent in units h = 1 with active cell i centred at i + 1/2; the
    child (h = 1/2) has its lower faces at parent faces F."""
    P = np.zeros((25,) + tuple(n + 2 * NG for n in np_[::-1]))
    C = np.zeros((25,) + tuple(n + 2 * NG for n in nc[::-1]))
    xp = [np.arange(n + 2 * NG) - NG + 0.5 for n in np_]
    xc = [F[d] + (np.arange(nc[d] + 2 * NG) - NG + 0.5) / 2.0 for d in range(3)]
    return P, C, xp, xc, np_, nc, F


def _poly(x, y, z, deg):
    return (1.0 + 0.3 * x) ** deg * (0.7 - 0.2 * y) ** deg * (1.1 + 0.25 * z) ** deg + 0.5 * x * y - z


@pytest.mark.parametrize("deg,exact", [(5, True), (6, False)])
def test_prolongation_polynomial(oz, deg, exact):
    P, C, xp, xc, np_, nc, F = _parent_child()
    Zp, Yp, Xp = np.meshgrid(xp[2], xp[1], xp[0], indexing="ij")
    Zc, Yc, Xc = np.meshgrid(xc[2], xc[1], xc[0], indexing="ij")
    for f in range(25):
        P[f] = _poly(Xp, Yp, Zp, deg) * (1 + f)
    oz.prolong([None, P, None], [0.0, 1.0, 0.0], np_, NG, C, nc, NG, F)
    want = np.stack([_poly(Xc, Yc, Zc, deg) * (1 + f) for f in range(25)])
    ghost = ~np.pad(np.ones(nc[::-1], bool), NG)
    err = np.abs(C[:, ghost] - want[:, ghost]).max() / np.abs(want[:, ghost]).max()
    if exact:
        assert err < 1e-13, err
        assert np.all(C[:, ~ghost] == 0.0)  # active child cells untouched
    else:
        assert err > 1e-9, err


def test_prolongation_time_levels(oz):
    """Three parent time levels of a field quadratic in time: the weights
    of theta reproduce its value at theta exactly."""
    P, C, xp, xc, np_, nc, F = _parent_child()
    Zp, Yp, Xp = np.meshgrid(xp[2], xp[1], xp[0], indexing="ij")
    base = _poly(Xp, Yp, Zp, 2)
    levels = [np.ascontiguousarray(np.broadcast_to(base * (1 + 0.4 * t + 0.3 * t * t), P.shape)) for t in (-1, 0, 1)]
    theta = 0.75
    wt, *_ = oz.transfer_weights(theta, 1)
    oz.prolong(levels, wt, np_, NG, C, nc, NG, F)
    Zc, Yc, Xc = np.meshgrid(xc[2], xc[1], xc[0], indexing="ij")
    want = _poly(Xc, Yc, Zc, 2) * (1 + 0.4 * theta + 0.3 * theta ** 2)
    ghost = ~np.pad(np.ones(nc[::-1], bool), NG)
    assert np.abs(C[:, ghost] - want[ghost]).max() < 1e-13 * np.abs(want).max()


def test_restriction_cubic(oz):
    P, C, xp, xc, np_, nc, F = _parent_child()
    Zc, Yc, Xc = np.meshgrid(xc[2], xc[1], xc[0], indexing="ij")
    for f in range(25):
        C[f] = _poly(Xc, Yc, Zc, 3) + f
    P[:] = -7.0
    oz.restrict(C, nc, NG, P, np_, NG, F)
    Zp, Yp, Xp = np.meshgrid(xp[2], xp[1], xp[0], indexing="ij")
    cov = np.zeros(P.shape[1:], bool)
    cov[NG + F[2]:NG + F[2] + nc[2] // 2, NG + F[1]:NG + F[1] + nc[1] // 2, NG + F[0]:NG + F[0] + nc[0] // 2] = True
    for f in range(25):
        want = _poly(Xp, Yp, Zp, 3) + f
        assert np.abs(P[f][cov] - want[cov]).max() < 1e-13 * np.abs(want[cov]).max()
    assert np.all(P[:, ~cov] == -7.0)  # only covered parent cells change


def _hierarchy(nlev=3, n=24, h0=1.0, bc0=I.BC_PERIODIC):
    """Boxes of n^3 cells centred on the origin, h halving per level; the
    child's lower faces sit at parent active cell n/4."""
    grids, Fs = [], []
    for lev in range(nlev):
        h = h0 / 2 ** lev
        grids.append(I.centered_grid(n, h, bc=bc0 if lev == 0 else I.BC_COPY))
        Fs.append((0, 0, 0) if lev == 0 else (n // 4,) * 3)
    return grids, Fs


def test_flat_space_stays_flat(oz):
    grids, Fs = _hierarchy()
    levels = [oz.Level(g, I.flat_state(g), F) for g, F in zip(grids, Fs)]
    oz.bo_advance(levels, 0.5, 2)
    for L in levels:
        assert np.array_equal(L.u, I.flat_state(L.grid))


def test_linear_gauge_drift_exact(oz):
    """beta^i = beta0^i + 0.75 B^i t with constant B and eta = 0 (no other
    field moves): every level, ghosts included, holds the exact value after
    each coarse step, in the first step (linear time interpolation) and the
    second (quadratic)."""
    grids, Fs = _hierarchy()
    B = np.array([0.02, -0.01, 0.015])
    b0 = np.array([0.1, 0.05, -0.03])
    levels = []
    for g, F in zip(grids, Fs):
        u = I.flat_state(g)
        for a in range(3):
            u[19 + a] = b0[a]
            u[22 + a] = B[a]
        levels.append(oz.Level(g, u, F))
    p = oz.params(eta=0.0)
    dt0 = 0.5
    for step in (1, 2):
        oz.bo_advance(levels, dt0, 1, p)
        t = step * dt0
        for lev, L in enumerate(levels):
            want = I.flat_state(L.grid)
            for a in range(3):
                want[19 + a] = b0[a] + 0.75 * B[a] * t
                want[22 + a] = B[a]
            err = np.abs(L.u - want).max()
            assert err < 1e-15, (step, lev, err)


def test_parent_covered_cells_are_restricted_child(oz):
    grids, Fs = _hierarchy(nlev=2, n=24)
    levels = []
    for g, F in zip(grids, Fs):
        u = I.flat_state(g) + 1e-3 * (I.random_strong_field_state(g, seed=3) - I.flat_state(g))
        levels.append(oz.Level(g, u, F))
    # child data must agree with the parent's where they overlap at t = 0:
    # start the child from the parent by prolongation of all its cells
    oz.bo_advance(levels, 0.25, 1)
    P, C = levels
    n = C.grid.n
    Pr = P.u.copy()
    oz.restrict(C.u, n, NG, Pr, P.grid.n, NG, C.F)
    assert np.array_equal(Pr, P.u)
