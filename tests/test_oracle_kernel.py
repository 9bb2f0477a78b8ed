"""Pins of the oracle's kernel and self term (P1), and of the generator's kernel table."""
import numpy as np
import pytest
from scipy import integrate

from oracle import kernel as ok


@pytest.mark.parametrize("h,k", [(0.5 / 12, 2 * np.pi), (4.0 / 64, 2 * np.pi), (0.3, 2 * np.pi), (0.05, 7.3)])
def test_self_integral_vs_quadrature(h, k):
    V = h ** 3
    a = ok.sphere_radius(V)
    # integral of g over the ball = int_0^a 4 pi r^2 g(r) dr
    f_re = lambda r: (4 * np.pi * r * r * ok.green(r, k)).real
    f_im = lambda r: (4 * np.pi * r * r * ok.green(r, k)).imag
    re, _ = integrate.quad(f_re, 0.0, a, epsabs=0, epsrel=2e-14, limit=200)
    im, _ = integrate.quad(f_im, 0.0, a, epsabs=0, epsrel=2e-14, limit=200)
    ref = re + 1j * im
    got = ok.self_integral(V, k)
    assert abs(got - ref) <= 1e-13 * abs(ref)


@pytest.mark.parametrize("h,k", [(0.5 / 12, 2 * np.pi), (4.0 / 64, 2 * np.pi), (2.0 / 48, 2 * np.pi), (0.02, 1.0)])
def test_self_integral_vs_taylor_series(h, k):
    """int_0^a r exp(-jkr) dr = sum_n (-jk)^n a^(n+2) / (n! (n+2)); leading term a^2/2 (static limit)."""
    from math import factorial
    V = h ** 3
    a = ok.sphere_radius(V)
    ser = sum((-1j * k) ** n * a ** (n + 2) / (factorial(n) * (n + 2)) for n in range(30))
    got = ok.self_integral(V, k)
    # the closed form cancels to order (ka)^2; its rounding error is ~1e-16 / (ka)^2 relative
    tol = 1e-15 / (k * a) ** 2 + 1e-15
    assert abs(got - ser) <= tol * abs(ser)
    assert abs(ser - a * a / 2) <= 1.0 * k * a * abs(ser)    # static limit a^2/2 dominates for small ka


def test_sphere_volume():
    V = 0.37
    a = ok.sphere_radius(V)
    assert abs(4.0 / 3.0 * np.pi * a ** 3 - V) <= 1e-15 * V


def test_green_properties():
    r = np.linspace(0.01, 3.0, 200)
    g = ok.green(r, 2 * np.pi)
    assert np.allclose(np.abs(g), 1 / (4 * np.pi * r), rtol=1e-14)
    # phase advances by -k r (exp(+j omega t) convention)
    assert np.allclose(np.angle(g * 4 * np.pi * r), np.angle(np.exp(-1j * 2 * np.pi * r)), atol=1e-12)


def test_dense_G_symmetric_and_self_term():
    G = ok.dense_G((3, 4, 2), 0.1, 2 * np.pi)
    assert np.array_equal(G, G.T)
    assert np.allclose(np.diag(G), ok.self_integral(1e-3, 2 * np.pi) / 1e-3, rtol=1e-15)


def test_generator_table_matches_closed_form():
    import h2gen
    g = h2gen.cube(6, 0.5, 4.0)
    tab = g.green_table()
    d2 = np.arange(1, tab.size)
    ref = ok.green(g.h * np.sqrt(d2.astype(float)), g.k)
    assert np.allclose(tab[1:], ref, rtol=1e-14, atol=0)
    assert abs(tab[0] - ok.self_integral(g.volume, g.k) / g.volume) <= 1e-14 * abs(tab[0])
