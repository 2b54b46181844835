"""Right-hand side of the constrained-realization system (oracle).
TEST INFRASTRUCTURE ONLY.

Sect. 2.3 prints b = P^T N^-1 d + P^T N^-1/2 omega_1 + S^-1 omega_2.  For x
to be a draw from the Gaussian posterior the covariance of b must equal A,
which fixes the last term as S^-1/2 omega_2 (the printed S^-1 is read as a
typo; the test suite pins the reading by K K^T = A with
K = [P^T N^-1/2, S^-1/2]).  omega = 0 gives the Wiener filter (mean).

    b = sum_nu P_nu^T (tau_nu d_nu + sqrt(tau_nu) omega_1,nu) + C^-1/2 omega_2
"""
import numpy as np

from . import philox
from .sht import lm_arrays


def build_rhs(model, d=None, omega1=None, omega2=None):
    """d, omega1: lists of band maps (or None); omega2: component vector or None."""
    b = np.zeros(model.n)
    for nu, band in enumerate(model.bands):
        tau = np.asarray(band["tau"], dtype=np.float64)
        f = np.zeros(band["grid"].npix)
        have = False
        if d is not None and d[nu] is not None:
            f = f + tau * np.asarray(d[nu], dtype=np.float64)
            have = True
        if omega1 is not None and omega1[nu] is not None:
            f = f + np.sqrt(tau) * np.asarray(omega1[nu], dtype=np.float64)
            have = True
        if have:
            b = b + model.project_t(f, nu)
    if omega2 is not None:
        parts = []
        for c, w in zip(model.comps, model.split(omega2)):
            ell = lm_arrays(c["lmax"])[0]
            parts.append(np.sqrt(c["invcl"][ell]) * w)
        b = b + model.join(parts)
    return b


def draw_omegas(model, seed, rhs=0):
    """omega_1 per band pixel and omega_2 per coefficient from Philox."""
    om1 = [philox.normals(seed, philox.STREAM_OMEGA1_BASE + nu, rhs, b["grid"].npix)
           for nu, b in enumerate(model.bands)]
    om2 = philox.normals(seed, philox.STREAM_OMEGA2, rhs, model.n)
    return om1, om2
