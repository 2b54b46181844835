"""Mask-restricted preconditioner M_mask and M_add = M_PI + M_mask (oracle).
TEST INFRASTRUCTURE ONLY.

Sect. 4.2, eq:M_mask:  M_mask = Z^T (Z S^-1 Z^T)^-1 Z, where Z is spherical
harmonic synthesis followed by selection of the pixels inside the mask.
Sect. 4.3, eq:rl: Z includes a low-pass filter, Z = (select) Y R with
R = diag(r_l), r_l = exp(-beta l^2 (l+1)^2) and beta such that r_{L/2}^2 = 0.05.
Sect. 4.4, eq:W: the inner system is G = Z S^-1 Z^T = Y D Y^T on the masked
pixels, D = diag(d_l), d_l = r_l^2 / C_l.  It is approximately inverted by a
multigrid V-cycle (fig:code:mg):
  * levels: HEALPix grids with Nside_H = Nside_h / 2; a coarse pixel belongs
    to the level's mask when all four of its children do; recursion stops at
    the first level with fewer than 1000 masked pixels (the bottom), which is
    solved by a pseudo-inverse G_h^+ of the dense G_h;
  * band-limits L_H = L_h / 2; restriction I_h^H = Y_H R_H Y_h^T W_h with R_H a
    Gaussian band-limited at L_H; coarse operator D_H = R_H^2 D_h;
  * smoother M_h = omega diag(G_h)^-1 with omega = 0.2 (diag(G_h) is one
    constant, sum_l d_l (2l+1) / 4 pi, since G_h is a rotation-invariant
    kernel evaluated at pixel centres);
  * the optimized V-cycle of fig:code:mg with J = Y_h^T W_h Y_h (Y_h
    synthesising to the masked pixels only) taken as I, as the paper does in
    its experiments: six SHTs per level; J can be applied exactly for the
    pins (exact_j=True), in which case the cycle equals the textbook
    Basic-V-cycle.
M_add = M_PI + M_mask (Sect. 4.2).  Several components: M_mask acts on each
component with its own prior (the mask-restricted system is block diagonal
in the components since S is); components or multipoles without prior
(C^-1 = 0) have d_l = 0.

Readings where the paper is silent (listed with the design notes):
  * the mask grid is a HEALPix grid (the paper's choice for the mixing maps);
    the mask itself is an input (True = masked);
  * the level-0 band-limit is the component's L_k;
  * r_l uses l = L/2 as a real number in r_{L/2}^2 = 0.05;
  * R_H: Gaussian b_l = exp(-l(l+1) sigma^2 / 2) whose FWHM is the coarse
    pixel size sqrt(4 pi / Npix_H), zero above L_H = floor(L_h / 2);
  * the bottom pseudo-inverse drops eigenvalues below rcond * max eigenvalue.
The HEALPix parent of a pixel is the coarse pixel containing its centre:
ang2pix in the RING scheme (Gorski et al. 2005) at Nside / 2.
"""
import math

import numpy as np

from . import geometry, sht


# ---------------------------------------------------------------- HEALPix
def ang2pix_ring(nside, z, phi):
    """RING-scheme pixel index of the points (z = cos theta, phi), Gorski et
    al. 2005: equatorial zone |z| <= 2/3 by the two edge-line indices, polar
    caps by the distance to the pole."""
    z = np.asarray(z, dtype=np.float64)
    phi = np.mod(np.asarray(phi, dtype=np.float64), 2.0 * math.pi)
    ns = int(nside)
    tt = phi / (0.5 * math.pi)  # in [0, 4)
    za = np.abs(z)
    out = np.empty(z.shape, dtype=np.int64)
    eq = za <= 2.0 / 3.0
    # equatorial zone
    t1 = ns * (0.5 + tt[eq])
    t2 = ns * z[eq] * 0.75
    jp = np.floor(t1 - t2).astype(np.int64)  # ascending edge line
    jm = np.floor(t1 + t2).astype(np.int64)  # descending edge line
    ir = ns + 1 + jp - jm                    # ring counted from z = 2/3, 1 .. 2 ns + 1
    kshift = 1 - (ir & 1)
    ip = (jp + jm - ns + kshift + 1) // 2
    ip = np.mod(ip, 4 * ns)
    out[eq] = 2 * ns * (ns - 1) + (ir - 1) * 4 * ns + ip
    # polar caps
    pc = ~eq
    tp = tt[pc] - np.floor(tt[pc])
    tmp = ns * np.sqrt(3.0 * (1.0 - za[pc]))
    jp = np.floor(tp * tmp).astype(np.int64)
    jm = np.floor((1.0 - tp) * tmp).astype(np.int64)
    ir = jp + jm + 1                         # ring counted from the nearest pole
    ip = np.floor(tt[pc] * ir).astype(np.int64)
    ip = np.mod(ip, 4 * ir)
    north = z[pc] > 0
    out[pc] = np.where(north, 2 * ir * (ir - 1) + ip, 12 * ns * ns - 2 * ir * (ir + 1) + ip)
    return out


def parents(nside):
    """RING index at Nside / 2 of the parent of every pixel at Nside."""
    g = geometry.healpix(nside)
    z, phi = g.pixel_centres()
    return ang2pix_ring(nside // 2, z, phi)


# ------------------------------------------------------------- filters
def lowpass_r(lmax):
    """r_l = exp(-beta l^2 (l+1)^2) with r_{L/2}^2 = 0.05 (eq:rl)."""
    h = 0.5 * lmax
    beta = math.log(20.0) / (2.0 * h * h * (h + 1.0) ** 2) if lmax > 0 else 0.0
    l = np.arange(lmax + 1, dtype=np.float64)
    return np.exp(-beta * l * l * (l + 1.0) ** 2)


def restriction_r(nside_coarse, lmax_coarse):
    """Gaussian whose FWHM is the coarse pixel size, zero above L_H."""
    fwhm = math.sqrt(4.0 * math.pi / (12.0 * nside_coarse * nside_coarse))
    sig = fwhm / math.sqrt(8.0 * math.log(2.0))
    l = np.arange(lmax_coarse + 1, dtype=np.float64)
    return np.exp(-0.5 * l * (l + 1.0) * sig * sig)


# ------------------------------------------------------------ levels
class Level:
    def __init__(self, nside, lmax, idx):
        self.nside = nside
        self.lmax = lmax
        self.grid = geometry.healpix(nside)
        self.idx = np.asarray(idx, dtype=np.int64)  # masked pixels (RING order)
        self.w = 4.0 * math.pi / self.grid.npix
        self.rH = None      # restriction filter to the next level (length L_H + 1)
        self.gplus = None   # bottom: pseudo-inverse per component


def hierarchy(nside, mask, lmax, nbottom=1000):
    """Levels from the mask grid down to the first level with fewer than
    nbottom masked pixels (or an odd Nside, or a band-limit below 2)."""
    mask = np.asarray(mask, dtype=bool)
    levels = [Level(nside, lmax, np.flatnonzero(mask))]
    while (len(levels[-1].idx) >= nbottom and levels[-1].nside >= 2 and levels[-1].nside % 2 == 0
           and levels[-1].lmax >= 2):
        h = levels[-1]
        ns_c = h.nside // 2
        par = parents(h.nside)
        cover = np.zeros(12 * ns_c * ns_c, dtype=np.int64)
        np.add.at(cover, par[h.idx], 1)
        Lc = h.lmax // 2
        h.rH = restriction_r(ns_c, Lc)
        levels.append(Level(ns_c, Lc, np.flatnonzero(cover == 4)))
    return levels


def level_d(levels, invcl):
    """d_l per level: d_0 = r_l^2 C_l^-1 (eq:W), d_H = r_H^2 d_h."""
    L0 = levels[0].lmax
    ic = np.zeros(L0 + 1)
    n = min(L0 + 1, len(invcl))
    ic[:n] = invcl[:n]
    d = [lowpass_r(L0) ** 2 * ic]
    for h in levels[:-1]:
        Lc = len(h.rH) - 1
        d.append(h.rH ** 2 * d[-1][:Lc + 1])
    return d


def legendre_p(lmax, x):
    """P_l(x) for l = 0..lmax (Bonnet's recurrence), shape [lmax+1, *x.shape]."""
    x = np.asarray(x, dtype=np.float64)
    P = np.empty((lmax + 1,) + x.shape)
    P[0] = 1.0
    if lmax >= 1:
        P[1] = x
    for l in range(2, lmax + 1):
        P[l] = ((2 * l - 1) * x * P[l - 1] - (l - 1) * P[l - 2]) / l
    return P


def dense_g(level, d):
    """G = Y D Y^T on the level's masked pixels by the addition theorem:
    G_ij = sum_l d_l (2l + 1) / (4 pi) P_l(n_i . n_j)."""
    z, phi = level.grid.pixel_centres()
    z, phi = z[level.idx], phi[level.idx]
    st = np.sqrt(np.maximum(0.0, (1.0 - z) * (1.0 + z)))
    v = np.stack([st * np.cos(phi), st * np.sin(phi), z], axis=1)
    cosg = np.clip(v @ v.T, -1.0, 1.0)
    L = len(d) - 1
    P = legendre_p(L, cosg)
    coef = np.asarray(d) * (2.0 * np.arange(L + 1) + 1.0) / (4.0 * math.pi)
    return np.tensordot(coef, P, axes=1)


def pinv_sym(G, rcond):
    """Pseudo-inverse of a symmetric matrix: eigenvalues below rcond * max
    |eigenvalue| are dropped."""
    ev, V = np.linalg.eigh(G)
    top = np.abs(ev).max() if len(ev) else 0.0
    keep = np.abs(ev) > rcond * top
    return (V[:, keep] / ev[keep]) @ V[:, keep].T


# ------------------------------------------------------------- V-cycle
def _synth_masked(level, L, alm):
    """Y at band-limit L on the level's grid, keeping the masked pixels."""
    return sht.synth(level.grid, L, alm)[level.idx]


def _adjoint_masked(level, L, vals):
    """Y^T at band-limit L of a map that is zero outside the level's mask."""
    f = np.zeros(level.grid.npix)
    f[level.idx] = vals
    return sht.adjoint(level.grid, L, f)


def _scale_l(alm, L, fl):
    ell = sht.lm_arrays(L)[0]
    return fl[ell] * alm


class MaskMultigrid:
    """Approximate inverse of G = Z S^-1 Z^T for one component (fig:code:mg)."""

    def __init__(self, levels, invcl, omega=0.2, rcond=1e-6, exact_j=False):
        self.levels = levels
        self.d = level_d(levels, invcl)
        self.omega = omega
        self.exact_j = exact_j
        self.smooth = []
        for lev, d in zip(levels, self.d):
            diag = float(np.sum(d * (2.0 * np.arange(len(d)) + 1.0)) / (4.0 * math.pi))
            self.smooth.append(omega / diag if diag > 0 else 0.0)
        bottom = levels[-1]
        Gb = dense_g(bottom, self.d[-1])
        self.gplus = pinv_sym(Gb, rcond) if len(bottom.idx) else np.zeros((0, 0))

    def _j(self, lev, alm):
        """J = Y_h^T W_h Y_h with Y_h synthesis to the masked pixels only: it
        zeroes what falls outside the mask (exact_j)."""
        return lev.w * _adjoint_masked(lev, lev.lmax, _synth_masked(lev, lev.lmax, alm))

    def vcycle(self, h, b):
        lev = self.levels[h]
        if h == len(self.levels) - 1:
            return self.gplus @ b
        crs = self.levels[h + 1]
        Lh, LH = lev.lmax, crs.lmax
        d = self.d[h]
        Mh = self.smooth[h]
        x = Mh * b                                              # pre-smoothing
        u = _adjoint_masked(lev, Lh, x)                         # Y_h^T x            (L_h, N_h)
        Du = _scale_l(u, Lh, d)
        JDu = self._j(lev, Du) if self.exact_j else Du
        rt = lev.w * _adjoint_masked(lev, LH, b) - sht.repack(JDu, Lh, LH)  # (L_H, N_h)
        rH = _synth_masked(crs, LH, _scale_l(rt, LH, lev.rH))   # Y_H R_H r~          (L_H, N_H)
        cH = self.vcycle(h + 1, rH)
        ct = _scale_l(_adjoint_masked(crs, LH, cH), LH, lev.rH)  # R_H Y_H^T c_H     (L_H, N_H)
        x = x + lev.w * _synth_masked(lev, LH, ct)              # + W_h Y_h c~        (L_H, N_h)
        ctp = sht.repack(ct, LH, Lh)
        Jct = self._j(lev, ctp) if self.exact_j else ctp
        x = x + Mh * (b - _synth_masked(lev, Lh, _scale_l(u + Jct, Lh, d)))  # post  (L_h, N_h)
        return x

    def basic_vcycle(self, h, b):
        """The textbook Basic-V-cycle of fig:code:mg with dense G_h and
        I_h^H = Y_H R_H Y_h^T W_h (tiny sizes only; for the pins)."""
        lev = self.levels[h]
        if h == len(self.levels) - 1:
            return self.gplus @ b
        crs = self.levels[h + 1]
        Gh = dense_g(lev, self.d[h])
        Mh = self.smooth[h]
        x = Mh * b
        r = b - Gh @ x
        rH = _synth_masked(crs, crs.lmax, _scale_l(lev.w * _adjoint_masked(lev, crs.lmax, r), crs.lmax, lev.rH))
        cH = self.basic_vcycle(h + 1, rH)
        ch = lev.w * _synth_masked(lev, crs.lmax, _scale_l(_adjoint_masked(crs, crs.lmax, cH), crs.lmax, lev.rH))
        x = x + ch
        return x + Mh * (b - Gh @ x)


class MaskPrecond:
    """M_mask = sum_k Z_k^T V_k Z_k with V_k the V-cycle approximation of
    (Z S_k^-1 Z^T)^-1 and Z = (select) Y R at the component band-limit."""

    def __init__(self, model, nside, mask, omega=0.2, rcond=1e-6, nbottom=1000, exact_j=False):
        self.model = model
        self.comp = []
        for c in model.comps:
            lv = hierarchy(nside, mask, c["lmax"], nbottom)
            mg = MaskMultigrid(lv, c["invcl"], omega, rcond, exact_j)
            self.comp.append((lv, mg, lowpass_r(c["lmax"])))

    def __call__(self, r):
        out = []
        for (lv, mg, rl), rk, c in zip(self.comp, self.model.split(r), self.model.comps):
            L = c["lmax"]
            if not np.any(mg.d[0]) or len(lv[0].idx) == 0:
                out.append(np.zeros_like(rk))
                continue
            b = _synth_masked(lv[0], L, _scale_l(rk, L, rl))    # Z r_k
            cvec = mg.vcycle(0, b)
            out.append(_scale_l(_adjoint_masked(lv[0], L, cvec), L, rl))  # Z^T
        return self.model.join(out)


class AddPrecond:
    """M_add = M_PI + M_mask (Sect. 4.2)."""

    def __init__(self, pinv, mask_precond):
        self.pinv = pinv
        self.mask = mask_precond

    def __call__(self, r):
        return self.pinv(r) + self.mask(r)
