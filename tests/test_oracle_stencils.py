"""Pins of the oracle's finite-difference stencils (paper Sec. 2.2: 4th-order
centred differences, 4th-order upwinded advection with a bias that follows
the sign of the shift, 6th-order Kreiss-Oliger dissipation).

Checked against what the mathematics fixes: exactness on polynomials up to
the stencil's degree, 4th-order convergence on smooth data, the KO grid-mode
eigenvalue, and that the upwind bias is the stable (dissipative) one for the
advection term +beta d_x f that the right-hand side adds."""
import numpy as np
import pytest

H = 0.37


def _x(n=15):
    return (np.arange(n) - 7.0) * H + 0.11


@pytest.mark.parametrize("deg", range(0, 6))
def test_d1_exact_to_degree_4(oz, deg):
    x = _x()
    f = x ** deg
    d = oz.stencil_1d("d1", f, H)[3:-3]
    exact = deg * x[3:-3] ** (deg - 1) if deg else 0 * x[3:-3]
    err = np.abs(d - exact).max()
    if deg <= 4:
        assert err < 1e-11 * max(1, np.abs(exact).max())
    else:  # leading error -h^4 f^(5)/30 for x^5: -h^4 * 120 / 30
        np.testing.assert_allclose(d - exact, -4 * H ** 4, rtol=1e-9)


@pytest.mark.parametrize("deg", range(0, 7))
def test_d2_exact_to_degree_5(oz, deg):
    x = _x()
    f = x ** deg
    d = oz.stencil_1d("d2", f, H)[3:-3]
    exact = deg * (deg - 1) * x[3:-3] ** (deg - 2) if deg >= 2 else 0 * x[3:-3]
    if deg <= 5:
        assert np.abs(d - exact).max() < 1e-10 * max(1, np.abs(exact).max())
    else:  # leading error -h^4 f^(6)/90 for x^6: -h^4 * 720 / 90
        np.testing.assert_allclose(d - exact, -8 * H ** 4, rtol=1e-8)


@pytest.mark.parametrize("sign", [1.0, -1.0])
@pytest.mark.parametrize("deg", range(0, 6))
def test_upwind_exact_to_degree_4(oz, deg, sign):
    x = _x()
    f = x ** deg
    d = oz.stencil_1d("up", f, H, sign)[3:-3]
    exact = deg * x[3:-3] ** (deg - 1) if deg else 0 * x[3:-3]
    err = d - exact
    if deg <= 4:
        assert np.abs(err).max() < 1e-11 * max(1, np.abs(exact).max())
    else:  # lopsided 5-point leading error: +h^4 f^(5)/20 for either bias (odd-order term)
        np.testing.assert_allclose(err, 6 * H ** 4, rtol=1e-8)


@pytest.mark.parametrize("deg", range(0, 6))
def test_ko6_annihilates_degree_5(oz, deg):
    x = _x()
    d = oz.stencil_1d("ko", x ** deg, H)[3:-3]
    assert np.abs(d).max() < 1e-10 * max(1, np.abs(x ** deg).max())


def test_ko6_grid_mode(oz):
    f = (-1.0) ** np.arange(15)
    d = oz.stencil_1d("ko", f, H)[3:-3]
    np.testing.assert_array_equal(d, -64.0 * f[3:-3])
    # x^6: the 6th difference of a degree-6 monomial is 6! h^6
    x = _x()
    np.testing.assert_allclose(oz.stencil_1d("ko", x ** 6, H)[3:-3], 720 * H ** 6, rtol=1e-9)


@pytest.mark.parametrize("op,order_deriv", [("d1", 1), ("d2", 2), ("up", 1)])
def test_fourth_order_convergence(oz, op, order_deriv):
    errs = []
    for n in (32, 64, 128):
        h = 2 * np.pi / n
        x = (np.arange(n + 6) - 3) * h
        f = np.sin(x)
        exact = np.cos(x) if order_deriv == 1 else -np.sin(x)
        errs.append(np.abs(oz.stencil_1d(op, f, h)[3:-3] - exact[3:-3]).max())
    r = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(r > 3.8) and np.all(r < 4.3), r


def test_mixed_exact_on_tensor_polynomials(oz):
    hx, hy = 0.3, 0.45
    x = (np.arange(13) - 6.0) * hx + 0.2
    y = (np.arange(11) - 5.0) * hy - 0.1
    Y, X = np.meshgrid(y, x, indexing="ij")
    for a in range(5):
        for b in range(5):
            f = X ** a * Y ** b
            exact = a * b * X ** max(a - 1, 0) * Y ** max(b - 1, 0)
            d = oz.mixed_2d(f, hx, hy)[3:-3, 3:-3]
            assert np.abs(d - exact[3:-3, 3:-3]).max() < 1e-10 * max(1, np.abs(exact).max())


def _symbol(oz, op, theta, sign):
    """Complex symbol lambda(theta) of a 1-D operator at h = 1, from its action
    on cos and sin at a point where theta*j = 0."""
    j = np.arange(15) - 7.0
    c = oz.stencil_1d(op, np.cos(theta * j), 1.0, sign)[7]
    s = oz.stencil_1d(op, np.sin(theta * j), 1.0, sign)[7]
    return c + 1j * s


def test_upwind_bias_is_dissipative(oz):
    """For d_t f = beta D f (the advection term the right-hand side adds) the
    growth rate is Re(beta lambda).  With the bias chosen from the sign of
    beta it is <= 0 for every wavenumber; the opposite bias grows."""
    thetas = np.linspace(0.0, np.pi, 41)
    for beta in (+0.7, -0.7):
        good = np.array([(beta * _symbol(oz, "up", t, np.sign(beta))).real for t in thetas])
        bad = np.array([(beta * _symbol(oz, "up", t, -np.sign(beta))).real for t in thetas])
        assert good.max() <= 1e-12
        assert bad.max() > 0.5
    # and the centred operator is neutral (purely imaginary symbol)
    assert max(abs(_symbol(oz, "d1", t, 1.0).real) for t in thetas) < 1e-12
