"""Spherical harmonic synthesis Y and its literal transpose Y^T (oracle).
TEST INFRASTRUCTURE ONLY.

Sect. 2.1 defines Y as the map from harmonic coefficients to pixel values
and Y^T W as analysis; Sect. 3.2 stresses that the operator appearing in
A is the plain transpose Y^T (adjoint synthesis), not analysis.

Harmonic vectors use the real orthonormal basis of ``legendre`` packed
m-major: [m = 0: l = 0..L], then for m = 1..L the cosine block
[l = m..L] followed by the sine block [l = m..L]; (L+1)^2 entries in total.

Synthesis, ring by ring:
    F^c_m(r) = c_m sum_l lambda_lm(z_r) u^c_lm,  F^s_m(r) likewise,
    f(r, j)  = F^c_0(r) + sum_{m=1..L} [F^c_m(r) cos(m phi_rj) + F^s_m(r) sin(m phi_rj)],
with c_0 = 1, c_m = sqrt(2).  The phi sum is a naive DFT evaluated directly
for every m <= L, so rings with fewer than 2L+1 pixels alias exactly as the
dense matrix does; there is no folding code here.

The transpose swaps the order: H^c_m(r) = sum_j f(r,j) cos(m phi_rj),
H^s_m(r) = sum_j f(r,j) sin(m phi_rj), v^{c|s}_lm = c_m sum_r lambda_lm(z_r) H^{c|s}_m(r).
"""
import math

import numpy as np

from .legendre import LegendreSweep


def nalm(lmax):
    return (lmax + 1) * (lmax + 1)


def m_offset(lmax, m):
    """Start of the m block in the packed layout (cosine part for m >= 1)."""
    if m == 0:
        return 0
    return (lmax + 1) + 2 * ((m - 1) * (lmax + 1) - (m - 1) * m // 2)


def index(lmax, l, m, part):
    """Packed index of (l, m, part), part 0 = cosine, 1 = sine."""
    if not (0 <= m <= l <= lmax):
        raise IndexError((l, m, lmax))
    if m == 0:
        if part != 0:
            raise IndexError("m = 0 has no sine part")
        return l
    return m_offset(lmax, m) + part * (lmax - m + 1) + (l - m)


def lm_arrays(lmax):
    """(ell, m, part) for every packed index."""
    ell = np.empty(nalm(lmax), dtype=np.int64)
    mm = np.empty_like(ell)
    part = np.empty_like(ell)
    ell[: lmax + 1] = np.arange(lmax + 1)
    mm[: lmax + 1] = 0
    part[: lmax + 1] = 0
    for m in range(1, lmax + 1):
        o = m_offset(lmax, m)
        n = lmax - m + 1
        for p in (0, 1):
            s = slice(o + p * n, o + (p + 1) * n)
            ell[s] = np.arange(m, lmax + 1)
            mm[s] = m
            part[s] = p
    return ell, mm, part


def _as2d(a):
    a = np.asarray(a, dtype=np.float64)
    return (a[None, :], True) if a.ndim == 1 else (a, False)


def _mlist(lmax, ms):
    """The m values to evaluate: all of 0..lmax, or a sorted subset (m above
    lmax carry no coefficients and are dropped)."""
    if ms is None:
        return list(range(lmax + 1))
    out = sorted(set(int(m) for m in ms))
    if out and out[0] < 0:
        raise ValueError("negative m")
    return [m for m in out if m <= lmax]


def _phase_from_alm(grid, lmax, alm, ms=None):
    """F^c, F^s of shape [nmaps, nring, lmax+1] (the Legendre half of Y)."""
    nmaps = alm.shape[0]
    Fc = np.zeros((nmaps, grid.nring, lmax + 1))
    Fs = np.zeros((nmaps, grid.nring, lmax + 1))
    sweep = LegendreSweep(grid.z, grid.sint, lmax)
    for m in _mlist(lmax, ms):
        sweep.skip_to(m)
        lam = sweep.table(m)  # [nring, lmax-m+1]
        n = lmax - m + 1
        if m == 0:
            Fc[:, :, 0] = alm[:, 0:n] @ lam.T
        else:
            o = m_offset(lmax, m)
            c = math.sqrt(2.0)
            Fc[:, :, m] = c * (alm[:, o:o + n] @ lam.T)
            Fs[:, :, m] = c * (alm[:, o + n:o + 2 * n] @ lam.T)
    return Fc, Fs


def synth(grid, lmax, alm, ms=None):
    """Y alm: pixel maps [nmaps, npix] (or [npix] for a 1-D input).

    ms (optional): evaluate only these m; the other m blocks of alm are taken
    as zero (the sum over m simply leaves them out)."""
    alm, squeeze = _as2d(alm)
    if alm.shape[1] != nalm(lmax):
        raise ValueError("alm has the wrong length for lmax")
    Fc, Fs = _phase_from_alm(grid, lmax, alm, ms)
    out = np.zeros((alm.shape[0], grid.npix))
    msel = np.array(_mlist(lmax, ms), dtype=np.int64)
    for r in range(grid.nring):
        phi = grid.ring_phi(r)
        arg = np.outer(phi, msel)
        o, n = grid.offset[r], grid.nphi[r]
        out[:, o:o + n] = Fc[:, r, msel] @ np.cos(arg).T + Fs[:, r, msel] @ np.sin(arg).T
    return out[0] if squeeze else out


def adjoint(grid, lmax, maps, ms=None):
    """Y^T maps: harmonic vectors [nmaps, (lmax+1)^2].

    ms (optional): compute only the outputs of these m (the other m blocks of
    the result are left zero)."""
    maps, squeeze = _as2d(maps)
    if maps.shape[1] != grid.npix:
        raise ValueError("map has the wrong number of pixels")
    nmaps = maps.shape[0]
    msel = np.array(_mlist(lmax, ms), dtype=np.int64)
    Hc = np.zeros((nmaps, grid.nring, lmax + 1))
    Hs = np.zeros((nmaps, grid.nring, lmax + 1))
    for r in range(grid.nring):
        phi = grid.ring_phi(r)
        arg = np.outer(phi, msel)
        o, n = grid.offset[r], grid.nphi[r]
        f = maps[:, o:o + n]
        Hc[:, r, msel] = f @ np.cos(arg)
        Hs[:, r, msel] = f @ np.sin(arg)
    out = np.zeros((nmaps, nalm(lmax)))
    sweep = LegendreSweep(grid.z, grid.sint, lmax)
    for m in msel:
        m = int(m)
        sweep.skip_to(m)
        lam = sweep.table(m)
        n = lmax - m + 1
        if m == 0:
            out[:, 0:n] = Hc[:, :, 0] @ lam
        else:
            o = m_offset(lmax, m)
            c = math.sqrt(2.0)
            out[:, o:o + n] = c * (Hc[:, :, m] @ lam)
            out[:, o + n:o + 2 * n] = c * (Hs[:, :, m] @ lam)
    return out[0] if squeeze else out


def analysis(grid, lmax, maps):
    """Y^T W maps (spherical harmonic analysis, Sect. 2.1)."""
    return adjoint(grid, lmax, np.asarray(maps) * grid.pixel_weights())


def repack(src, lsrc, ldst):
    """Copy coefficients between packed layouts of different band-limits;
    entries with l > min(lsrc, ldst) are dropped or zero-filled."""
    src, squeeze = _as2d(src)
    out = np.zeros((src.shape[0], nalm(ldst)))
    lc = min(lsrc, ldst)
    for m in range(lc + 1):
        n = lc - m + 1
        if m == 0:
            out[:, 0:n] = src[:, 0:n]
        else:
            so, do_ = m_offset(lsrc, m), m_offset(ldst, m)
            out[:, do_:do_ + n] = src[:, so:so + n]
            out[:, do_ + ldst - m + 1:do_ + ldst - m + 1 + n] = \
                src[:, so + lsrc - m + 1:so + lsrc - m + 1 + n]
    return out[0] if squeeze else out
