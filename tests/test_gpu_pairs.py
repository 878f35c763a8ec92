"""GPU hierarchy with patch pairs (moving levels of Sec. 2.2.1, Fig. 1: one
patch per tracked object at each moving depth, all patches of a depth in one
launch per stage, exchange where they overlap, restriction into every coarse
patch they cover) against the oracle's patch hierarchy on the same seeded
data; plus its exact cases: the constant-B gauge drift on overlapping pairs,
bitwise pi symmetry of a pair that is its own mirror (graph replay equal to
direct launches), and far-apart chains that evolve like single chains."""
import numpy as np
import pytest

from gpu_helpers import normrel, to_host
from paper_2607_08743_amd import inputs as I
from paper_2607_08743_amd import z4c

pytestmark = pytest.mark.gpu
TOL = 1e-12
CENTERS = [(-1.0, 0.0, 0.0), (1.0, 0.0, 0.0)]


def _pt(centers=CENTERS, moving=(24, 16), root_n=32, bc0=I.BC_PERIODIC):
    return I.pair_hierarchy(root_n, 1.0, centers, moving, bc0=bc0)


def _states(pt, seed, amp=1e-3, beta=None):
    out = []
    for q, (g, *_) in enumerate(pt):
        u = I.flat_state(g) + amp * (I.random_strong_field_state(g, seed=seed + q) - I.flat_state(g))
        if beta is not None:
            u[19:22] += np.asarray(beta)[:, None, None, None]
        out.append(u)
    return out


def _gpu(pt, states, dt0, nsteps, xp=None, params=None, use_graph=True, tile=None):
    H = z4c.Hierarchy([(g, u, F, p, o) for (g, F, p, o), u in zip(pt, states)], dt0, params=params, tile=tile)
    if xp is not None:
        H.set_moving(xp)
    H.advance(nsteps, use_graph=use_graph)
    x, F, x0 = H.puncture()
    got = [to_host(u) for u in H.u]
    H.close()
    return got, x, F, x0


def _oracle(oz, pt, states, dt0, nsteps, xp=None, p=None, perturb=None):
    lv = []
    for (g, F, par, o), u in zip(pt, states):
        v = u.copy()
        if perturb is not None:
            v = v + np.spacing(v) * perturb.choice([-1.0, 1.0], size=v.shape)
        lv.append(oz.Level(g, v, F, parent=par, obj=o))
    x = None
    if xp is None:
        oz.bo_advance(lv, dt0, nsteps, p)
    else:
        x = oz.bo_advance_moving(lv, xp, dt0, nsteps, p)
    return lv, x


def _compare(got, lv, alt):
    for q, (a, L, c) in enumerate(zip(got, lv, alt)):
        m = L.grid.active_mask()
        e = normrel(a, L.u, m)
        sens = normrel(c.u, L.u, m)
        print(f"patch {q} normrel max {e.max():.2e} (oracle 1-ulp sensitivity max {sens.max():.2e})")
        assert np.all(e <= np.maximum(TOL, 20 * sens)), (q, e)
        assert np.abs(a[:, m] - L.u[:, m]).max() <= TOL * np.abs(L.u[:, m]).max()


def test_pair_parity(oz):
    print("case: pair hierarchy (root 32^3, pairs 24^3 and 16^3), 2 root steps vs oracle", flush=True)
    pt = _pt()
    st = _states(pt, seed=40)
    got, *_ = _gpu(pt, st, 0.5, 2, use_graph=False)
    lv, _ = _oracle(oz, pt, st, 0.5, 2)
    alt, _ = _oracle(oz, pt, st, 0.5, 2, perturb=np.random.default_rng(1))
    _compare(got, lv, alt)
    g2, *_ = _gpu(pt, st, 0.5, 2, use_graph=True)
    for a, b in zip(got, g2):
        assert np.array_equal(a, b)


def test_pair_moving_parity(oz):
    """Both objects move (constant shift added to the data) and cross the
    shift thresholds: punctures, patch placement and states after 3 root
    steps against the oracle.  The shift stays small: near |beta| = 0.5 on
    these data (lapse near 1) Courant 0.5 is past the stability limit of RK4
    with KO dissipation and rounding differences grow 100-fold per unit time
    in any implementation."""
    print("case: moving pair vs oracle, 3 root steps", flush=True)
    beta = np.array([0.2, -0.125, 0.075])
    pt = _pt()
    st = _states(pt, seed=50, beta=beta)
    xp = np.array(CENTERS) + np.array([[-0.45, 0.3, 0.1], [0.45, -0.3, -0.1]])
    got, x, F, x0 = _gpu(pt, st, 0.5, 3, xp=xp)
    lv, xr = _oracle(oz, pt, st, 0.5, 3, xp=xp)
    alt, _ = _oracle(oz, pt, st, 0.5, 3, xp=xp, perturb=np.random.default_rng(2))
    print("punctures gpu", x.tolist(), "oracle", xr.tolist())
    assert np.abs(x - xr).max() <= 1e-12
    assert any(F[q] != pt[q][1] for q in range(1, 5))  # a patch moved
    for q, L in enumerate(lv):
        assert F[q] == L.F and np.allclose(x0[q], L.grid.x0, rtol=0, atol=1e-14), q
    _compare(got, lv, alt)


def test_pair_linear_gauge_drift_exact():
    print("case: pair hierarchy constant-B shift drift, exact", flush=True)
    B = np.array([0.02, -0.01, 0.015])
    b0 = np.array([0.1, 0.05, -0.03])
    pt = _pt()
    st = []
    for g, *_ in pt:
        u = I.flat_state(g)
        u[19:22] = b0[:, None, None, None]
        u[22:25] = B[:, None, None, None]
        st.append(u)
    H = z4c.Hierarchy([(g, u, F, p, o) for (g, F, p, o), u in zip(pt, st)], 0.5,
                      params=z4c.default_params(eta=0.0))
    for step in (1, 2, 3):
        H.advance(1, use_graph=True)
        t = 0.5 * step
        for q, ((g, *_), u) in enumerate(zip(pt, H.u)):
            want = I.flat_state(g)
            want[19:22] = (b0 + 0.75 * B * t)[:, None, None, None]
            want[22:25] = B[:, None, None, None]
            m = g.active_mask()
            assert np.abs(to_host(u)[:, m] - want[:, m]).max() < 1e-15, (step, q)
    H.close()


def _mirror(u):
    return u[:, :, ::-1, ::-1] * I.PI_PARITY[:, None, None, None]


@pytest.mark.parametrize("tile_i", [0, -1])
def test_pair_pi_symmetry_bitwise(tile_i):
    """The pair at (-1, 0, 0), (1, 0, 0) is its own pi mirror: with patch B's
    data the mirror image of patch A's, every step keeps it so bit for bit
    (mirror-symmetric summation order in every transfer, commutative pair
    sums in the exchange and the restriction)."""
    print(f"case: pair pi symmetry, tile {tile_i}", flush=True)
    pt = _pt()
    st = _states(pt, seed=60)
    st[0] = I.pi_symmetrize(st[0])
    st[2] = _mirror(st[1])
    st[4] = _mirror(st[3])
    tile = z4c.tiles(z4c.FP64)[tile_i]
    got, *_ = _gpu(pt, st, 0.5, 3, use_graph=True, tile=tile)
    assert np.array_equal(got[0], _mirror(got[0]))
    assert np.array_equal(got[2], _mirror(got[1]))
    assert np.array_equal(got[4], _mirror(got[3]))
    assert not np.array_equal(got[1], st[1])
    eager, *_ = _gpu(pt, st, 0.5, 3, use_graph=False, tile=tile)
    for a, b in zip(got, eager):
        assert np.array_equal(a, b)


def test_far_pair_equals_single_chains():
    """Chains that do not meet: after the first root step each chain's
    patches are bitwise what a hierarchy holding that chain alone gives."""
    print("case: far pair vs single chains, bitwise", flush=True)
    far = [(-5.0, 0.0, 0.0), (5.0, 0.0, 0.0)]
    pt = _pt(centers=far, moving=(16, 8))
    st = _states(pt, seed=70)
    got, *_ = _gpu(pt, st, 0.5, 1)
    for o in (0, 1):
        chain = [0] + [q for q in range(1, 5) if pt[q][3] == o]
        sub = [(pt[q][0], st[q], pt[q][1], i - 1, -1) for i, q in enumerate(chain)]
        H = z4c.Hierarchy(sub, 0.5)
        H.advance(1)
        for i, q in enumerate(chain[1:], 1):
            assert np.array_equal(to_host(H.u[i]), got[q]), (o, q)
        H.close()


def test_nine_patches_one_depth_parity(oz):
    """Nine 16^3 patches at one depth (a 3 x 3 layout in a 48^3 periodic
    root): 18 prolongation entries per parent step, more than one batch of
    the separable passes takes, against the oracle after 2 root steps."""
    print("case: nine patches at one depth vs oracle, 2 root steps", flush=True)
    root = I.centered_grid(48, 1.0, bc=I.BC_PERIODIC)
    pt = [(root, (0, 0, 0), -1, -1)]
    for a in range(3):
        for b in range(3):
            F = (8 + 11 * a, 8 + 11 * b, 20)
            x0 = tuple(root.x0[d] + (F[d] - 0.25) * root.h[d] for d in range(3))
            pt.append((I.Grid((16, 16, 16), (0.5,) * 3, x0, I.BC_COPY, 3), F, 0, -1))
    st = _states(pt, seed=90)
    got, *_ = _gpu(pt, st, 0.5, 2)
    lv, _ = _oracle(oz, pt, st, 0.5, 2)
    alt, _ = _oracle(oz, pt, st, 0.5, 2, perturb=np.random.default_rng(5))
    _compare(got, lv, alt)
