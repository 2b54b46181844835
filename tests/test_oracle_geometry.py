"""Pins for the oracle's grids (HEALPix RING, Gauss-Legendre)."""
import math
import os

import numpy as np
import pytest

from oracle import geometry

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_healpix_low_resolution_rings_match_published_layout():
    rows = np.loadtxt(os.path.join(GOLD, "healpix_ring_centres.txt"))
    for nside in (1, 2):
        g = geometry.healpix(nside)
        sel = rows[rows[:, 0] == nside]
        assert g.nring == len(sel)
        np.testing.assert_allclose(g.z, sel[:, 2], atol=1e-15)
        np.testing.assert_array_equal(g.nphi, sel[:, 3].astype(int))
        np.testing.assert_allclose(g.phi0 / math.pi, sel[:, 4], atol=1e-15)


@pytest.mark.parametrize("nside", [1, 2, 3, 4, 8, 13, 64])
def test_healpix_invariants(nside):
    g = geometry.healpix(nside)
    assert g.npix == 12 * nside * nside
    assert g.nring == 4 * nside - 1
    # north/south mirror symmetry of rings
    np.testing.assert_allclose(g.z, -g.z[::-1], atol=1e-15)
    np.testing.assert_array_equal(g.nphi, g.nphi[::-1])
    np.testing.assert_allclose(g.phi0, g.phi0[::-1], atol=0)
    # sin(theta) consistent with z and accurate near the poles
    np.testing.assert_allclose(g.sint ** 2 + g.z ** 2, 1.0, atol=1e-14)
    # equal-area pixels: cumulative pixel count above ring i equals the
    # area fraction north of the boundary between rings (pixel centres sit
    # half a pixel row inside), checked at the cap/belt boundary ring.
    # polar cap |z| > 2/3 covers 1/6 of the sphere: the rings above the
    # transition ring plus half of that ring hold exactly Npix / 6 pixels.
    ncap = int(g.nphi[:nside - 1].sum()) + g.nphi[nside - 1] // 2
    assert ncap * 6 == g.npix
    assert abs(g.z[nside - 1] - 2.0 / 3.0) < 1e-15
    # pixel weights sum to the sphere area
    assert abs(g.pixel_weights().sum() - 4 * math.pi) < 1e-12
    # mean z over pixel centres vanishes, mean z^2 tends to 1/3
    z, phi = g.pixel_centres()
    assert abs(z.mean()) < 1e-15
    assert abs((z * z).mean() - 1.0 / 3.0) < 0.5 / nside ** 2 + 1e-15


@pytest.mark.parametrize("n", [1, 2, 5, 17, 33, 64])
def test_gauss_legendre_matches_numpy(n):
    x, w = geometry.gauss_legendre_nodes(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xr[::-1], atol=3e-16)
    # numpy's weights are themselves good to ~1e-12 at n = 64
    np.testing.assert_allclose(w, wr[::-1], rtol=2e-11)


@pytest.mark.parametrize("n", [5, 33])
def test_gauss_legendre_weights_high_precision(n):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    x, w = geometry.gauss_legendre_nodes(n)
    for i in range(n):
        r = mpmath.findroot(lambda t: mpmath.legendre(n, t), x[i])
        d = mpmath.diff(lambda t: mpmath.legendre(n, t), r)
        assert abs(float(r) - x[i]) < 2e-16
        assert abs(float(2 / ((1 - r ** 2) * d ** 2)) / w[i] - 1) < 1e-12


def test_gauss_legendre_grid_weights_integrate_polynomials():
    g = geometry.gauss_legendre(9, 19)
    z, phi = g.pixel_centres()
    w = g.pixel_weights()
    # integral over the sphere of z^k cos(j phi): exact up to degree 17 / 9
    for k in range(0, 18):
        exact = 0.0 if k % 2 else 4 * math.pi / (k + 1)
        assert abs(w @ z ** k - exact) < 1e-13
    for j in range(1, 10):
        assert abs(w @ np.cos(j * phi)) < 1e-13


def test_gauss_legendre_polar_weights_at_large_n():
    """At n = 1001 the nodes nearest the poles sit where P_{n-1}(x) is steep
    in x; their weights must still be right to about 1e-12 relative (the
    formula evaluated at a rounded x is off by ~1e-7 there).  Reference:
    Newton on P_n and the weight 2 (1 - x^2) / (n P_{n-1}(x))^2, all in
    60-digit decimal arithmetic."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    n = 1001
    x, w = geometry.gauss_legendre_nodes(n)

    def p_pair(xd):
        p0, p1 = Decimal(1), xd
        for j in range(2, n + 1):
            p0, p1 = p1, ((2 * j - 1) * xd * p1 - (j - 1) * p0) / j
        return p1, p0

    for k in (0, 1, n // 3, n // 2, n - 2, n - 1):
        xd = Decimal(repr(float(x[k])))
        for _ in range(8):
            pn, pm = p_pair(xd)
            xd -= pn / (n * (xd * pn - pm) / (xd * xd - 1))
        pn, pm = p_pair(xd)
        wd = 2 * (1 - xd * xd) / (n * pm) ** 2
        assert abs(float(xd) - x[k]) < 2e-16, k
        assert abs(float((Decimal(repr(float(w[k]))) - wd) / wd)) < 1e-12, k
