"""Normalised associated Legendre functions (oracle).  TEST INFRASTRUCTURE ONLY.

lambda_{l m}(z) is the latitude part of the real orthonormal spherical
harmonics used for every harmonic vector (the paper works with (L+1)^2
real coefficients per component, Sect. 3.3; the basis itself is a reading
recorded with the design notes):

    Y_{l0} = lambda_{l0},  Y^c_{lm} = sqrt(2) lambda_{lm} cos(m phi),
    Y^s_{lm} = sqrt(2) lambda_{lm} sin(m phi),        no Condon-Shortley sign,

so that sum over m of the squares obeys the addition theorem.  The functions
follow the textbook three-term recurrence in l at fixed m:

    lambda_00      = 1 / sqrt(4 pi)
    lambda_mm      = sqrt((2m+1) / (2m)) sin(theta) lambda_{m-1,m-1}
    lambda_{m+1,m} = sqrt(2m+3) z lambda_mm
    lambda_lm      = a_lm (z lambda_{l-1,m} - b_lm lambda_{l-2,m})
    a_lm = sqrt((4 l^2 - 1) / (l^2 - m^2)),
    b_lm = sqrt(((l-1)^2 - m^2) / (4 (l-1)^2 - 1)).

lambda_mm ~ sin^m(theta) leaves the float64 range near the poles at large m,
so the start value and the recurrence carry an explicit power-of-two
exponent per ring; the value handed back is the exact function rounded once
to float64 (tiny values become subnormal or zero at that final rounding).
Nothing is truncated or skipped.
"""
import math

import numpy as np

_RESCALE = 2.0 ** 600
_RESCALE_EXP = 600


def recurrence_coefficients(m, lmax):
    """a_lm and b_lm for l = m .. lmax (entries for l < m+2 are unused)."""
    l = np.arange(m, lmax + 1, dtype=np.float64)
    a = np.zeros(lmax - m + 1)
    b = np.zeros(lmax - m + 1)
    if lmax >= m + 1:
        a[1] = math.sqrt(2.0 * m + 3.0)
    if lmax >= m + 2:
        ll = l[2:]
        a[2:] = np.sqrt((4.0 * ll * ll - 1.0) / (ll * ll - m * m))
        b[2:] = np.sqrt(((ll - 1.0) ** 2 - m * m) / (4.0 * (ll - 1.0) ** 2 - 1.0))
    return a, b


class LegendreSweep:
    """Yields lambda_{l m}(z_r) for m = 0, 1, ..., lmax in order.

    ``table(m)`` must be called with m increasing by one each time; it
    returns an array of shape [nring, lmax - m + 1] (column j is l = m + j).
    The start value lambda_mm is carried from m - 1 to m as mantissa and
    exponent, so no intermediate ever underflows.
    """

    def __init__(self, z, sint, lmax):
        self.z = np.asarray(z, dtype=np.float64)
        self.sint = np.asarray(sint, dtype=np.float64)
        self.lmax = int(lmax)
        n = len(self.z)
        self._mant = np.full(n, 1.0 / math.sqrt(4.0 * math.pi))
        self._exp = np.zeros(n, dtype=np.int64)
        self._m = -1

    def _advance_start(self):
        self._m += 1
        m = self._m
        if m > 0:
            self._mant = self._mant * (math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * self.sint)
            mant, e = np.frexp(self._mant)
            self._mant = mant
            self._exp = self._exp + e.astype(np.int64)

    def skip_to(self, m):
        """Advance the carried start value so that the next table is for m."""
        while self._m + 1 < m:
            self._advance_start()

    def table(self, m):
        if m != self._m + 1:
            raise ValueError("LegendreSweep.table must be called with m = 0, 1, 2, ...")
        self._advance_start()
        lmax = self.lmax
        a, b = recurrence_coefficients(m, lmax)
        nring = len(self.z)
        out = np.zeros((nring, lmax - m + 1))
        mu_prev = np.zeros(nring)
        mu_cur = self._mant.copy()
        e = self._exp.copy()
        out[:, 0] = np.ldexp(mu_cur, e)
        for j in range(1, lmax - m + 1):
            if j == 1:
                mu_next = a[1] * self.z * mu_cur
            else:
                mu_next = a[j] * (self.z * mu_cur - b[j] * mu_prev)
            mu_prev, mu_cur = mu_cur, mu_next
            big = np.abs(mu_cur) > _RESCALE
            if np.any(big):
                mu_cur = np.where(big, mu_cur / _RESCALE, mu_cur)
                mu_prev = np.where(big, mu_prev / _RESCALE, mu_prev)
                e = np.where(big, e + _RESCALE_EXP, e)
            out[:, j] = np.ldexp(mu_cur, e)
        return out


def lambda_lm(z, sint, l, m):
    """lambda_{l m} at the given points (convenience; runs the full sweep)."""
    sw = LegendreSweep(np.atleast_1d(z), np.atleast_1d(sint), l)
    for mm in range(m):
        sw.table(mm)
    return sw.table(m)[:, l - m]
