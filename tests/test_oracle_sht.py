"""Pins for the oracle's Legendre functions and spherical harmonic transforms."""
import math

import numpy as np
import pytest
import scipy.special as sps

from oracle import dense, geometry, sht
from oracle.legendre import LegendreSweep, lambda_lm


def test_legendre_closed_forms():
    th = np.array([0.01, 0.7, 1.5707963267948966, 2.2, 3.1])
    z, s = np.cos(th), np.sin(th)
    np.testing.assert_allclose(lambda_lm(z, s, 0, 0), 1 / math.sqrt(4 * math.pi), rtol=1e-15)
    np.testing.assert_allclose(lambda_lm(z, s, 1, 0), math.sqrt(3 / (4 * math.pi)) * z, rtol=1e-15)
    np.testing.assert_allclose(lambda_lm(z, s, 1, 1), math.sqrt(3 / (8 * math.pi)) * s, rtol=1e-15)
    np.testing.assert_allclose(lambda_lm(z, s, 2, 0),
                               math.sqrt(5 / (4 * math.pi)) * 0.5 * (3 * z * z - 1), rtol=1e-13)


def test_legendre_matches_scipy():
    """scipy includes the Condon-Shortley sign; the basis here does not."""
    th = np.array([1e-3, 0.05, 0.4, 1.1, 1.5707963267948966, 2.0, 3.0])
    z, s = np.cos(th), np.sin(th)
    L = 150
    sw = LegendreSweep(z, s, L)
    worst = 0.0
    for m in range(L + 1):
        tab = sw.table(m)
        for l in range(m, L + 1, 7):
            ref = (-1) ** m * sps.sph_legendre_p(l, m, th)
            ref = np.asarray(ref).reshape(-1)
            scale = max(1e-300, float(np.max(np.abs(ref))))
            worst = max(worst, float(np.max(np.abs(tab[:, l - m] - ref))) / scale)
    assert worst < 1e-12


def _lambda_high_precision(l, m, theta):
    """|lambda_lm(cos theta)| from the explicit polynomial form
    P_l^m(x) = (1-x^2)^(m/2) 2^-l sum_k (-1)^k C(l,k) C(2l-2k,l) (l-2k)!/(l-2k-m)! x^(l-2k-m)
    with integer coefficients, summed at a precision that survives the
    cancellation (mpmath)."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = int(1.6 * l) + 100
    x = mpmath.cos(mpmath.mpf(theta))
    acc = mpmath.mpf(0)
    for k in range(0, (l - m) // 2 + 1):
        n = l - 2 * k
        c = math.comb(l, k) * math.comb(2 * l - 2 * k, l) * (math.factorial(n) // math.factorial(n - m))
        term = c * x ** (n - m)
        acc += -term if k % 2 else term
    p = (1 - x * x) ** (mpmath.mpf(m) / 2) * acc / mpmath.mpf(2) ** l
    norm = mpmath.sqrt((2 * l + 1) / (4 * mpmath.pi) * mpmath.factorial(l - m)
                       / mpmath.factorial(l + m))
    return abs(norm * p)


@pytest.mark.parametrize("l,m,theta", [(2000, 300, 0.05), (1500, 900, 0.45),
                                       (600, 590, 0.9), (2500, 1800, 0.5)])
def test_legendre_deep_start_matches_high_precision(l, m, theta):
    """lambda_mm underflows float64 here; the exponent-carrying start must
    still give the right representable lambda_lm."""
    import mpmath
    assert (math.sin(theta) ** m) < 1e-300 or m > 500  # start really is out of range
    ref = _lambda_high_precision(l, m, theta)
    z, s = math.cos(theta), math.sin(theta)
    got = abs(lambda_lm(np.array([z]), np.array([s]), l, m)[0])
    if ref < mpmath.mpf("1e-300"):
        assert got < 1e-290
    else:
        # evaluating at the rounded float64 point costs ~ l^2 * 1e-16
        assert abs(got / float(ref) - 1) < 1e-16 * l * l + 1e-13, (got, float(ref))


def test_addition_theorem_high_l_near_poles():
    """sum_m over the real basis of Y_lm^2 = (2l+1)/(4 pi) at every point."""
    th = np.array([2e-4, 3e-3, 0.05, 0.8, 1.5, 2.9, math.pi - 1e-3])
    z, s = np.cos(th), np.sin(th)
    L = 700
    sw = LegendreSweep(z, s, L)
    acc = np.zeros((len(th), L + 1))
    for m in range(L + 1):
        t = sw.table(m)
        acc[:, m:] += (1.0 if m == 0 else 2.0) * t * t
    ell = np.arange(L + 1)
    # near the poles the rounded float64 point costs ~ l^2 eps relative
    np.testing.assert_allclose(acc, np.broadcast_to((2 * ell + 1) / (4 * math.pi), acc.shape),
                               rtol=1e-10)


def test_packed_layout():
    L = 7
    seen = set()
    for l in range(L + 1):
        for m in range(l + 1):
            for p in ((0,) if m == 0 else (0, 1)):
                seen.add(sht.index(L, l, m, p))
    assert seen == set(range(sht.nalm(L)))
    ell, mm, part = sht.lm_arrays(L)
    for i in range(sht.nalm(L)):
        assert sht.index(L, ell[i], mm[i], part[i]) == i


def _real_sh_scipy(lmax, theta, phi):
    Y = np.zeros((len(theta), sht.nalm(lmax)))
    for l in range(lmax + 1):
        for m in range(l + 1):
            c = sps.sph_harm_y(l, m, theta, phi) * (-1) ** m
            if m == 0:
                Y[:, sht.index(lmax, l, 0, 0)] = c.real
            else:
                Y[:, sht.index(lmax, l, m, 0)] = math.sqrt(2) * c.real
                Y[:, sht.index(lmax, l, m, 1)] = math.sqrt(2) * c.imag
    return Y


@pytest.mark.parametrize("spec,lmax", [(("healpix", 4), 16), (("gl", 9, 17), 8)])
def test_dense_y_matches_scipy(spec, lmax):
    g = geometry.make_grid(spec)
    z, phi = g.pixel_centres()
    Y = dense.dense_y(g, lmax)
    Yr = _real_sh_scipy(lmax, np.arccos(z), phi)
    assert np.max(np.abs(Y - Yr)) < 1e-12


@pytest.mark.parametrize("spec,lmax", [(("healpix", 4), 16), (("healpix", 3), 13),
                                       (("gl", 9, 17), 8), (("gl", 6, 7), 9)])
def test_ring_synthesis_equals_dense(spec, lmax):
    """Ring-wise synthesis (naive DFT, aliasing where Nphi < 2L+1) equals the
    dense matrix built by direct evaluation."""
    g = geometry.make_grid(spec)
    rng = np.random.default_rng(5)
    a = rng.standard_normal((2, sht.nalm(lmax)))
    Y = dense.dense_y(g, lmax)
    np.testing.assert_allclose(sht.synth(g, lmax, a), a @ Y.T, atol=1e-12)
    f = rng.standard_normal((2, g.npix))
    np.testing.assert_allclose(sht.adjoint(g, lmax, f), f @ Y, atol=1e-12)


@pytest.mark.parametrize("nrings,nphi,lmax", [(33, 65, 32), (17, 33, 16), (5, 9, 4)])
def test_gauss_legendre_round_trip_exact(nrings, nphi, lmax):
    """Y^T W Y = I when the GL grid supports the band-limit (Sect. 2.1)."""
    g = geometry.gauss_legendre(nrings, nphi)
    rng = np.random.default_rng(1)
    a = rng.standard_normal(sht.nalm(lmax))
    back = sht.analysis(g, lmax, sht.synth(g, lmax, a))
    assert np.max(np.abs(back - a)) < 1e-13
    if lmax <= 16:
        Y = dense.dense_y(g, lmax)
        G = Y.T @ (g.pixel_weights()[:, None] * Y)
        assert np.max(np.abs(G - np.eye(len(G)))) < 1e-13


def test_gauss_legendre_round_trip_fails_beyond_band_limit():
    g = geometry.gauss_legendre(9, 19)
    Y = dense.dense_y(g, 10)
    G = Y.T @ (g.pixel_weights()[:, None] * Y)
    assert np.max(np.abs(G - np.eye(len(G)))) > 1e-3


def test_adjoint_identity_healpix_aliasing():
    g = geometry.healpix(8)
    L = 40  # > 2 * Nside: polar rings alias
    rng = np.random.default_rng(3)
    x = rng.standard_normal(sht.nalm(L))
    y = rng.standard_normal(g.npix)
    lhs = sht.synth(g, L, x) @ y
    rhs = x @ sht.adjoint(g, L, y)
    assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(y))


def test_healpix_round_trip_is_approximate():
    """On HEALPix Y^T W Y is close to, but not exactly, I (Sect. 3.2, App. A.1)."""
    g = geometry.healpix(8)
    Y = dense.dense_y(g, 16)
    G = Y.T @ (g.pixel_weights()[:, None] * Y)
    ev = np.linalg.eigvalsh(G)
    assert 0.7 < ev.min() and ev.max() < 1.3
    assert np.max(np.abs(G - np.eye(len(G)))) > 1e-6


def test_repack_round_trip():
    rng = np.random.default_rng(0)
    a = rng.standard_normal(sht.nalm(9))
    b = sht.repack(a, 9, 14)
    assert np.array_equal(sht.repack(b, 14, 9), a)
    ell = sht.lm_arrays(14)[0]
    assert np.all(b[ell > 9] == 0)
