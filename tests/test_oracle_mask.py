"""Pins for the oracle's mask-restricted preconditioner (Sect. 4.2-4.4,
fig:code:mg): HEALPix pixel lookup and hierarchy, the dense inner system by
brute force, the filters' defining values, the reorganised V-cycle against
the textbook one, symmetry and convergence of the cycle, and M_mask itself
against its dense definition when the hierarchy has a single level."""
import math

import numpy as np
import pytest

from oracle import dense, geometry, mask, sht
from oracle.model import Model
from paper_1710_00621_amd import inputs


@pytest.mark.parametrize("nside", [1, 2, 3, 4, 8, 16, 32])
def test_ang2pix_ring_round_trip(nside):
    """Every pixel centre (RING geometry pinned against the published ring
    layout) maps back to its own index."""
    g = geometry.healpix(nside)
    z, phi = g.pixel_centres()
    np.testing.assert_array_equal(mask.ang2pix_ring(nside, z, phi), np.arange(g.npix))


@pytest.mark.parametrize("nside", [2, 4, 8, 16, 32])
def test_parents_four_children_each_nearby(nside):
    par = mask.parents(nside)
    assert np.bincount(par, minlength=3 * nside * nside).tolist() == [4] * (3 * nside * nside)
    gf, gc = geometry.healpix(nside), geometry.healpix(nside // 2)

    def vec(g):
        z, phi = g.pixel_centres()
        st = np.sqrt((1 - z) * (1 + z))
        return np.stack([st * np.cos(phi), st * np.sin(phi), z], axis=1)

    vf, vc = vec(gf), vec(gc)
    # each child centre is closer to its parent's centre than the coarse pixel size
    ang = np.arccos(np.clip(np.sum(vf * vc[par], axis=1), -1, 1))
    assert ang.max() < math.sqrt(4 * math.pi / gc.npix)


def test_dense_g_equals_y_d_yt():
    """G = Y D Y^T on the masked pixels (addition theorem) against the dense Y
    evaluated pixel by pixel."""
    lev = mask.Level(8, 12, np.arange(0, 768, 5))
    d = np.abs(np.random.default_rng(0).standard_normal(13))
    G = mask.dense_g(lev, d)
    Y = dense.dense_y(lev.grid, 12)[lev.idx]
    ell = sht.lm_arrays(12)[0]
    np.testing.assert_allclose(G, (Y * d[ell]) @ Y.T, atol=1e-13 * np.abs(G).max())


def test_filters_defining_values():
    for L in (16, 64, 2000):
        r = mask.lowpass_r(L)
        assert abs(r[L // 2] ** 2 - 0.05) < 1e-12  # r_{L/2}^2 = 0.05 (eq:rl)
        assert r[0] == 1.0 and np.all(np.diff(r) <= 0)
    # Gaussian of FWHM = coarse pixel size: ln b_l = -l(l+1) FWHM^2 / (16 ln 2)
    ns, L = 8, 16
    fwhm2 = 4 * math.pi / (12 * ns * ns)
    l = np.arange(L + 1)
    np.testing.assert_allclose(np.log(mask.restriction_r(ns, L)), -l * (l + 1) * fwhm2 / (16 * math.log(2)),
                               rtol=1e-13, atol=1e-15)


def _levels(nside=16, lmax=32, nbottom=100):
    g = geometry.healpix(nside)
    z, phi = g.pixel_centres()
    m = (np.abs(z) < 0.35) | ((z > 0.7) & (np.cos(phi) > 0.2))
    return mask.hierarchy(nside, m, lmax, nbottom=nbottom)


def _invcl(L):
    return inputs.inv_cl("cmb", L)


def test_smoother_is_omega_over_diagonal_of_g():
    lv = _levels()
    mg = mask.MaskMultigrid(lv, _invcl(32))
    for lev, d, s in zip(lv, mg.d, mg.smooth):
        G = mask.dense_g(lev, d)
        np.testing.assert_allclose(0.2 / np.diag(G), s, rtol=1e-12)


def test_hierarchy_levels_and_coverage():
    lv = _levels()
    assert [(l.nside, l.lmax) for l in lv] == [(16, 32), (8, 16), (4, 8)][:len(lv)]
    assert len(lv) >= 2 and len(lv[-1].idx) < 100 <= len(lv[-2].idx)
    for h, H in zip(lv[:-1], lv[1:]):
        # a coarse masked pixel has all four children masked
        par = mask.parents(h.nside)
        fine = np.zeros(h.grid.npix, dtype=bool)
        fine[h.idx] = True
        for p in H.idx:
            assert fine[par == p].all()


def test_optimized_cycle_with_exact_j_equals_basic_cycle():
    """fig:code:mg: the reorganised cycle (restriction and interpolation sharing
    SHTs with G_h) equals the textbook Basic-V-cycle when J is applied."""
    lv = _levels()
    mg = mask.MaskMultigrid(lv, _invcl(32), exact_j=True)
    b = np.random.default_rng(1).standard_normal(len(lv[0].idx))
    x1, x2 = mg.vcycle(0, b), mg.basic_vcycle(0, b)
    np.testing.assert_allclose(x1, x2, atol=1e-12 * np.abs(x2).max())
    # J taken as I is a controlled approximation of the same cycle
    x3 = mask.MaskMultigrid(lv, _invcl(32)).vcycle(0, b)
    assert 0 < np.abs(x3 - x2).max() / np.abs(x2).max() < 0.2


def test_basic_cycle_symmetric_and_convergent():
    lv = _levels(8, 16, 40)
    mg = mask.MaskMultigrid(lv, _invcl(16), exact_j=True, rcond=1e-12)
    n = len(lv[0].idx)
    V = np.stack([mg.basic_vcycle(0, e) for e in np.eye(n)], axis=1)
    np.testing.assert_allclose(V, V.T, atol=1e-10 * np.abs(V).max())
    # as a stationary iteration on G x = b (b in the range of G) the error
    # shrinks in the G norm
    G = mask.dense_g(lv[0], mg.d[0])
    xt = np.random.default_rng(2).standard_normal(n)
    b = G @ xt
    x = np.zeros(n)
    errs = []
    for _ in range(6):
        x = x + mg.basic_vcycle(0, b - G @ x)
        e = x - xt
        errs.append(float(e @ G @ e))
    assert errs[-1] < 0.5 * errs[0] and all(a >= b_ * (1 - 1e-9) for a, b_ in zip(errs, errs[1:]))


def test_single_level_m_mask_matches_dense_definition():
    """With fewer masked pixels than the bottom size the hierarchy is one level
    and M_mask = Z^T G^+ Z exactly, Z = (masked rows of Y) R, G = Z S^-1 Z^T
    (eq:M_mask, eq:rl, eq:W); two components, each with its own prior."""
    g = geometry.healpix(8)
    z, phi = g.pixel_centres()
    m = np.abs(z) < 0.25
    L = 12
    comps = [{"lmax": L, "invcl": inputs.inv_cl("cmb", L)},
             {"lmax": L, "invcl": inputs.inv_cl("powerlaw", L)}]
    bands = [{"grid": g, "lmax": L, "beam": np.ones(L + 1), "tau": np.ones(g.npix)}]
    mdl = Model(bands, comps, np.array([[1.0, 0.5]]))
    Mm = mask.MaskPrecond(mdl, 8, m, rcond=1e-6)
    assert len(Mm.comp[0][0]) == 1
    r = np.random.default_rng(3).standard_normal(mdl.n)
    got = Mm(r)
    Y = dense.dense_y(g, L)[m]
    ell = sht.lm_arrays(L)[0]
    rl = mask.lowpass_r(L)[ell]
    Z = Y * rl
    ref = []
    for c, rk in zip(comps, mdl.split(r)):
        G = (Z * c["invcl"][ell]) @ Z.T
        ev, V = np.linalg.eigh(G)
        keep = np.abs(ev) > 1e-6 * np.abs(ev).max()
        Gp = (V[:, keep] / ev[keep]) @ V[:, keep].T
        ref.append(Z.T @ (Gp @ (Z @ rk)))
    ref = np.concatenate(ref)
    np.testing.assert_allclose(got, ref, atol=1e-10 * np.abs(ref).max())
