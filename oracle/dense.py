"""Dense builders for tiny band-limits (oracle).  TEST INFRASTRUCTURE ONLY.

Y is written out as a matrix by evaluating every real spherical harmonic
at every pixel centre (Sect. 2.1: Y maps coefficients to pixel values), and
A = S^-1 + sum_nu P_nu^T diag(tau_nu) P_nu (eq:A) is assembled from it with
P_nu = Y_nu B_nu q_{nu,k} (eq:P with scalar mixing).  Only for L <= ~32.
"""
import math

import numpy as np

from . import sht
from .legendre import LegendreSweep


def dense_y(grid, lmax):
    """Y as a [npix, (lmax+1)^2] matrix, by direct evaluation per pixel."""
    z, phi = grid.pixel_centres()
    sint = np.repeat(grid.sint, grid.nphi)  # accurate sin(theta) per pixel
    Y = np.zeros((grid.npix, sht.nalm(lmax)))
    sweep = LegendreSweep(z, sint, lmax)
    for m in range(lmax + 1):
        lam = sweep.table(m)
        n = lmax - m + 1
        if m == 0:
            Y[:, 0:n] = lam
        else:
            o = sht.m_offset(lmax, m)
            Y[:, o:o + n] = math.sqrt(2.0) * lam * np.cos(m * phi)[:, None]
            Y[:, o + n:o + 2 * n] = math.sqrt(2.0) * lam * np.sin(m * phi)[:, None]
    return Y


def dense_p(model, nu):
    """P_nu as a [npix_nu, n] matrix."""
    b = model.bands[nu]
    Yb = dense_y(b["grid"], b["lmax"])
    ell_b = sht.lm_arrays(b["lmax"])[0]
    YB = Yb * b["beam"][ell_b][None, :]
    P = np.zeros((b["grid"].npix, model.n))
    for k, c in enumerate(model.comps):
        # column map component layout -> band layout
        eye = np.eye(sht.nalm(c["lmax"]))
        R = sht.repack(eye, c["lmax"], b["lmax"])  # rows: comp idx, cols: band idx
        if (nu, k) in getattr(model, "mixing_maps", {}):
            # eq:Q: Q~ = Y^T W Q Y as a dense matrix on the pair's grid
            grid, qmap = model.mixing_maps[(nu, k)]
            Yg = dense_y(grid, c["lmax"])
            Qt = Yg.T @ ((grid.pixel_weights() * np.asarray(qmap))[:, None] * Yg)
            P[:, model.offsets[k]:model.offsets[k + 1]] = YB @ R.T @ Qt
        else:
            P[:, model.offsets[k]:model.offsets[k + 1]] = model.q[nu, k] * (YB @ R.T)
    return P


def dense_a(model):
    """A = S^-1 + sum_nu P_nu^T diag(tau_nu) P_nu."""
    A = np.diag(model.apply_prior_inv(np.ones(model.n)))
    for nu, b in enumerate(model.bands):
        P = dense_p(model, nu)
        A += P.T @ (b["tau"][:, None] * P)
    return A
