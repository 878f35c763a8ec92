"""Pins of the oracle's hierarchy under equatorial symmetry (an equatorial
root; patches whose lower z face is the symmetry plane read the parent's
layers below the plane as mirror images and mirror their own lower ghost
layers).

* The reflected prolongation reproduces, at every child ghost, polynomials of
  degree <= 5 per variable that are even in z (fields of even z parity) or
  odd in z (odd parity) from the parent's active cells alone: the parent's
  layers below the plane hold NaN and are never read.  Without the
  reflection the same geometry is refused.
* The half hierarchy (equatorial root, every patch on the plane) evolves like
  the upper half of the full hierarchy with z-symmetric data (Sommerfeld root,
  every patch centred on z = 0), whose evolution involves no reflection code:
  to rounding, since the oracle's stencil sums run in index order, which is
  not mirror-symmetric (a sign error in one parity gives O(1e-3)).
* Flat space stays exactly flat on every patch of the half hierarchy, and a
  pure gauge translation in the plane moves both punctures by -beta t exactly
  with z = 0 kept, the patches shifting in x only (one root step, before the
  outgoing boundary, which a constant shift does not satisfy, reaches them).
"""
import numpy as np
import pytest

from paper_2607_08743_amd import inputs as I

NG = 3


def _zpoly(X, Y, Z, odd):
    e = (1.0 + 0.3 * X) ** 5 * (0.7 - 0.2 * Y) ** 5 * (1.1 + 0.05 * Z * Z) ** 2 + 0.5 * X * Y
    return Z * e if odd else e


def test_reflected_prolongation_parity_polynomials(oz):
    np_, nc, F = (24, 22, 12), (16, 12, 8), (4, 5, 0)
    P = np.zeros((25,) + tuple(n + 2 * NG for n in np_[::-1]))
    C = np.zeros((25,) + tuple(n + 2 * NG for n in nc[::-1]))
    xp = [np.arange(n + 2 * NG) - NG + 0.5 for n in np_]
    xc = [F[d] + (np.arange(nc[d] + 2 * NG) - NG + 0.5) / 2.0 for d in range(3)]
    Zp, Yp, Xp = np.meshgrid(xp[2], xp[1], xp[0], indexing="ij")
    Zc, Yc, Xc = np.meshgrid(xc[2], xc[1], xc[0], indexing="ij")
    odd = I.Z_PARITY < 0
    for f in range(25):
        P[f] = _zpoly(Xp, Yp, Zp, odd[f]) * (1 + 0.1 * f)
    P[:, :NG] = np.nan  # the layers below the plane are never read
    oz.prolong([None, P, None], [0.0, 1.0, 0.0], np_, NG, C, nc, NG, F, refl=True)
    ghost = ~np.pad(np.ones(nc[::-1], bool), NG)
    for f in range(25):
        want = _zpoly(Xc, Yc, Zc, odd[f]) * (1 + 0.1 * f)
        err = np.abs(C[f][ghost] - want[ghost]).max() / np.abs(want[ghost]).max()
        assert err < 1e-13, (f, err)
    with pytest.raises(RuntimeError):
        oz.prolong([None, P, None], [0.0, 1.0, 0.0], np_, NG, C, nc, NG, F, refl=False)


def _full(seed=11):
    pt = I.pair_hierarchy(32, 1.0, [(-2.0, 0.0, 0.0), (2.0, 0.0, 0.0)], (16,), fixed=(24,), bc0=I.BC_SOMMERFELD)
    st = []
    for q, (g, *_) in enumerate(pt):
        u = I.flat_state(g) + 1e-3 * (I.random_strong_field_state(g, seed=seed + q) - I.flat_state(g))
        st.append(I.z_symmetrize(u))
    return pt, st


def _levels(oz, pt, st):
    return [oz.Level(g, u.copy(), F, parent=p, obj=o) for (g, F, p, o), u in zip(pt, st)]


def test_half_hierarchy_matches_full(oz):
    from gpu_helpers import normrel
    pt, st = _full()
    hp, hs = I.upper_half_patches(pt, st)
    full = _levels(oz, pt, st)
    half = _levels(oz, hp, hs)
    oz.bo_advance(full, 0.5, 2)
    oz.bo_advance(half, 0.5, 2)
    for q, (F_, H_) in enumerate(zip(full, half)):
        m = H_.grid.active_mask()
        if q == 0:
            m[:] = True
            m[:NG] = False  # the mirrored layers are not evolved in the half box
        got = H_.u
        want = I.upper_half(F_.u, NG)
        e = normrel(got, want, m)
        assert e.max() < 1e-9, (q, e.max())
    assert not np.array_equal(half[1].u, hs[1])  # the data did evolve


def test_half_hierarchy_flat_exact(oz):
    """Flat space stays exactly flat on every patch: a field given the wrong
    z parity in a mirror fill or a reflected prolongation would turn its
    non-zero flat value (W, alpha, the diagonal of gt) into its negative."""
    pt, _ = _full()
    hp, _ = I.upper_half_patches(pt, [I.flat_state(g) for g, *_ in pt])
    lv = _levels(oz, hp, [I.flat_state(g) for g, *_ in hp])
    oz.bo_advance(lv, 0.5, 2)
    for L in lv:
        assert np.array_equal(L.u, I.flat_state(L.grid))


def test_plane_pair_translation_exact(oz):
    """A pure gauge translation in the plane, for one root step on a root
    wide enough that its outgoing boundary (which a constant shift does not
    satisfy) cannot reach the patches in that time: both punctures move by
    -beta dt0 exactly, z stays 0, the finest patch of each object shifts in x
    and the patches keep their state."""
    beta = np.array([0.4, -0.25, 0.0])
    pt = I.pair_hierarchy(48, 1.0, [(-2.0, 0.0, 0.0), (2.0, 0.0, 0.0)], (16,), fixed=(32,), bc0=I.BC_SOMMERFELD)
    hp, _ = I.upper_half_patches(pt, [I.flat_state(g) for g, *_ in pt])
    st = []
    for g, *_ in hp:
        u = I.flat_state(g)
        u[19:22] = beta[:, None, None, None]
        st.append(u)
    lv = _levels(oz, hp, st)
    xp0 = np.array([[-2.45, 0.3, 0.0], [2.45, -0.3, 0.0]])
    x = oz.bo_advance_moving(lv, xp0, 0.5, 1, oz.params(eta=0.0))
    assert np.abs(x - (xp0 - beta * 0.5)).max() < 1e-14, x
    assert np.abs(x[:, 2]).max() < 1e-30  # on the plane (beta_z vanishes there up to rounding)
    assert lv[2].F[0] == hp[2][1][0] - 1 and lv[2].F[1:] == hp[2][1][1:]  # object 0 (patch 2) moved in x only
    for L in lv[1:]:
        m = L.grid.active_mask()
        want = I.flat_state(L.grid)
        want[19:22] = beta[:, None, None, None]
        assert np.abs(L.u[:, m] - want[:, m]).max() < 1e-12
