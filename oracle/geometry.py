"""Ring grids on the sphere (oracle).  TEST INFRASTRUCTURE ONLY.

The paper uses HEALPix for the sky maps and recommends Gauss-Legendre (GL)
grids where an exact quadrature is wanted (Sect. 2.2, the paragraph under
eq:Q; Sect. 2.1 on Y^T W Y = I).  Neither healpy nor a grid library is used:
both grids are written out from their published definitions.

* HEALPix RING scheme (Gorski et al. 2005): rings i = 1 .. 4 Nside - 1.
  North cap (i < Nside): z = 1 - i^2 / (3 Nside^2), Nphi = 4 i,
  phi0 = pi / (4 i).  Belt (Nside <= i <= 3 Nside): z = 4/3 - 2 i / (3 Nside),
  Nphi = 4 Nside, phi0 = pi / (4 Nside) when (i - Nside) is even, else 0.
  South cap mirrors the north cap (z -> -z).  Pixel j of a ring sits at
  phi0 + 2 pi j / Nphi.  Quadrature weight: uniform 4 pi / Npix (the paper
  notes Y^T W is only approximate on HEALPix, Sect. 3.2).
* Gauss-Legendre: nodes are the roots of P_n ordered north to south
  (z descending), Nphi points per ring starting at phi = 0; pixel weight
  w_r * 2 pi / Nphi with w_r the GL weight.

Every ring carries z, sin(theta) evaluated without cancellation near the
poles, Nphi, phi0 and the offset of its first pixel.
"""
import math

import numpy as np


class Grid:
    """Plain container: per-ring arrays plus per-pixel weights."""

    def __init__(self, kind, z, sint, nphi, phi0, weight_per_ring, params):
        self.kind = kind
        self.z = np.asarray(z, dtype=np.float64)
        self.sint = np.asarray(sint, dtype=np.float64)
        self.nphi = np.asarray(nphi, dtype=np.int64)
        self.phi0 = np.asarray(phi0, dtype=np.float64)
        self.nring = len(self.z)
        self.offset = np.concatenate([[0], np.cumsum(self.nphi)[:-1]]).astype(np.int64)
        self.npix = int(self.nphi.sum())
        self.ring_weight = np.asarray(weight_per_ring, dtype=np.float64)
        self.params = params

    def pixel_weights(self):
        """Diagonal of W: one quadrature weight per pixel."""
        return np.repeat(self.ring_weight, self.nphi)

    def pixel_centres(self):
        """(z, phi) of every pixel in ring-major order."""
        z = np.repeat(self.z, self.nphi)
        phi = np.empty(self.npix)
        for r in range(self.nring):
            o, n = self.offset[r], self.nphi[r]
            phi[o:o + n] = self.phi0[r] + 2.0 * math.pi * np.arange(n) / n
        return z, phi

    def ring_phi(self, r):
        n = int(self.nphi[r])
        return self.phi0[r] + 2.0 * math.pi * np.arange(n) / n


def healpix(nside):
    """HEALPix RING geometry for a given Nside (any positive integer)."""
    if nside < 1:
        raise ValueError("nside must be >= 1")
    ns = nside
    nr = 4 * ns - 1
    z = np.empty(nr)
    sint = np.empty(nr)
    nphi = np.empty(nr, dtype=np.int64)
    phi0 = np.empty(nr)
    for k in range(nr):
        i = k + 1
        if i < ns or i > 3 * ns:
            ii = i if i < ns else 4 * ns - i
            one_minus = ii * ii / (3.0 * ns * ns)  # 1 - |z|
            zz = 1.0 - one_minus
            st = math.sqrt(one_minus * (2.0 - one_minus))
            z[k] = zz if i < ns else -zz
            sint[k] = st
            nphi[k] = 4 * ii
            phi0[k] = math.pi / (4.0 * ii)
        else:
            zz = 4.0 / 3.0 - 2.0 * i / (3.0 * ns)
            z[k] = zz
            sint[k] = math.sqrt((1.0 - zz) * (1.0 + zz))
            nphi[k] = 4 * ns
            phi0[k] = math.pi / (4.0 * ns) if (i - ns) % 2 == 0 else 0.0
    npix = 12 * ns * ns
    w = np.full(nr, 4.0 * math.pi / npix)
    return Grid("healpix", z, sint, nphi, phi0, w, {"nside": ns})


def _legendre_theta(n, th):
    """P_n(cos th) and P_{n-1}(cos th), vectorised over th.

    Bonnet's recurrence j P_j = (2j - 1) x P_{j-1} - (j - 1) P_{j-2}, rewritten
    with t = 1 - x = 2 sin^2(th/2) and the differences D_j = P_j - P_{j-1}:
        j D_j = (j - 1) D_{j-1} - (2j - 1) t P_{j-1}.
    Taking t from th (not from a rounded x) keeps full relative precision near
    the poles, where P_{n-1}(x) is steep in x.
    """
    t = 2.0 * np.sin(0.5 * th) ** 2
    if n == 0:
        return np.ones_like(th), np.zeros_like(th)
    prev = np.ones_like(th)
    p = 1.0 - t
    d = -t
    for j in range(2, n + 1):
        d = ((j - 1) * d - (2 * j - 1) * t * p) / j
        prev = p
        p = p + d
    return p, prev


def gauss_legendre_nodes(n, return_sint=False):
    """Roots of P_n (descending) and the GL weights.

    Newton iteration on theta for the roots with theta <= pi/2 (the others by
    the symmetry x -> -x), with P_n(cos theta) from _legendre_theta; at a root
    P_n' = n P_{n-1} / (1 - x^2), so w = 2 sin^2(theta) / (n P_{n-1})^2.
    """
    h = (n + 1) // 2
    k = np.arange(h)
    th = math.pi * (k + 0.75) / (n + 0.5)
    for _ in range(100):
        p, pm1 = _legendre_theta(n, th)
        # d/dtheta P_n(cos theta) = n (cos theta P_n - P_{n-1}) / sin theta
        dth = p * np.sin(th) / (n * (np.cos(th) * p - pm1))
        th = th - dth
        if np.max(np.abs(dth)) < 1e-16:
            break
    p, pm1 = _legendre_theta(n, th)
    xn = np.cos(th)
    if n % 2 == 1:
        xn[-1] = 0.0
    sn = np.sin(th)
    wn = 2.0 * sn * sn / (n * pm1) ** 2
    m = n // 2  # mirrored (southern) nodes
    x = np.concatenate([xn, -xn[:m][::-1]])
    w = np.concatenate([wn, wn[:m][::-1]])
    st = np.concatenate([sn, sn[:m][::-1]])
    return (x, w, st) if return_sint else (x, w)


def gauss_legendre(nrings, nphi):
    """GL grid: nrings rings at the GL nodes, nphi pixels per ring, phi0 = 0."""
    if nrings < 1 or nphi < 1:
        raise ValueError("nrings and nphi must be >= 1")
    x, w, sint = gauss_legendre_nodes(nrings, return_sint=True)
    ringw = w * 2.0 * math.pi / nphi
    return Grid("gl", x, sint, np.full(nrings, nphi, dtype=np.int64),
                np.zeros(nrings), ringw, {"nrings": nrings, "nphi": nphi})


def make_grid(spec):
    """Grid from a spec tuple: ("healpix", nside) or ("gl", nrings, nphi)."""
    if spec[0] == "healpix":
        return healpix(int(spec[1]))
    if spec[0] == "gl":
        return gauss_legendre(int(spec[1]), int(spec[2]))
    raise ValueError(f"unknown grid spec {spec!r}")
