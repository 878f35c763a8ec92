"""Pins of the oracle's equatorial-symmetry boundary (reflection z -> -z
across the lower z face, Sommerfeld on the other faces).

1. Its ghost fill against the parity rule written out here from the index
   structure of each field name: a component changes sign under z -> -z once
   per z index it carries.
2. The half box evolves bitwise like the upper half of the full box whose
   data are reflection-symmetric: the full box is a plain Sommerfeld box, so
   that evolution involves no reflection code at all.  Non-zero z-odd fields
   (shift, At_xz, Gt^z, ...) make a wrong sign in any parity visible.
"""
import numpy as np

from paper_2607_08743_amd import inputs as I


def _z_parity_from_names():
    out = []
    for name in I.FIELD_NAMES:
        idx = name.split("_", 1)[1] if "_" in name else ""
        out.append((-1.0) ** idx.count("z"))
    return np.array(out)


def _full_box(n=16, seed=5):
    """n^3 Sommerfeld box of extent 32, symmetric about z = 0 and about the z
    axis, holding Brill-Lindquist data plus a 1e-3 smooth perturbation in
    every field.  With n = 8 or 16 the cell centres are exact in binary, so
    the Sommerfeld terms see identical coordinates in the full and the half
    box."""
    g = I.centered_grid(n, 32.0 / n, bc=I.BC_SOMMERFELD)
    u = I.brill_lindquist_state(g)
    u = u + 1e-3 * (I.random_strong_field_state(g, seed=seed) - I.flat_state(g))
    return g, I.z_symmetrize(I.pi_symmetrize(u))


def _half_grid(g):
    n = g.n
    return I.Grid((n[0], n[1], n[2] // 2), g.h, (g.x0[0], g.x0[1], 0.5 * g.h[2]), I.BC_EQUATORIAL, g.ng)


def test_parity_table_matches_index_rule():
    assert np.array_equal(I.Z_PARITY, _z_parity_from_names())


def test_reflection_ghost_fill(oz):
    g, u = _full_box(12)
    gh = _half_grid(g)
    v = I.random_strong_field_state(gh, seed=11)
    before = v.copy()
    oz.apply_ghosts(v, gh.as_dict())
    ng = gh.ng
    par = _z_parity_from_names()
    for k in range(ng):
        assert np.array_equal(v[:, k], par[:, None, None] * before[:, 2 * ng - 1 - k]), k
    assert np.array_equal(v[:, ng:], before[:, ng:])  # nothing else touched


def test_half_box_evolves_like_full_box(oz):
    g, u = _full_box(16)
    assert np.array_equal(u, u[:, ::-1] * I.Z_PARITY[:, None, None, None])
    assert np.any(np.abs(u[21]) > 1e-5) and np.any(np.abs(u[10]) > 1e-5)  # z-odd fields are not zero
    gh = _half_grid(g)
    half = I.upper_half(u, g.ng)
    assert half.shape == gh.shape
    dt = 0.5 * g.h[0]
    full = u.copy()
    oz.rk4(full, g.as_dict(), dt, 2)
    oz.rk4(half, gh.as_dict(), dt, 2)
    # the full box stays exactly symmetric, and its upper half is the half box
    assert np.array_equal(full, full[:, ::-1] * I.Z_PARITY[:, None, None, None])
    assert np.array_equal(half, I.upper_half(full, g.ng))
    assert not np.array_equal(full, u)


def test_half_box_rhs_matches_full_box(oz):
    g, u = _full_box(16, seed=9)  # h = 2: cell centres are exact in both boxes
    gh = _half_grid(g)
    half = I.upper_half(u, g.ng)
    rf = oz.rhs(u, g.as_dict())
    rh = oz.rhs(half, gh.as_dict())
    ng = g.ng
    # evolved points of the half box: everything at and above the plane;
    # the mirrored layers below it carry no right-hand side
    assert np.array_equal(rh[:, ng:], I.upper_half(rf, ng)[:, ng:])
    assert np.all(rh[:, :ng] == 0.0)
