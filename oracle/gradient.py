"""Gradients of a Wiener-filter loss through the solve (oracle).
TEST INFRASTRUCTURE ONLY.

The solution x = A^-1 b of Sect. 2.3 (eq:A, b = sum_nu P_nu^T N_nu^-1 d_nu)
depends on the data maps d_nu and, through P_nu = Y_nu B_nu q_{nu,k}
(eq:P with Q~ = q I, Sect. 3.3), on the mixing scalars q.  For the loss

    L(d, q) = 1/2 x^T S^-1 x + sum_nu (d_nu - P_nu x)^T N_nu^-1 (d_nu - P_nu x)

the implicit-function gradient uses one extra solve with the symmetric A:

    g = dL/dx (explicit) = S^-1 x - 2 sum_nu P_nu^T N^-1 (d_nu - P_nu x),
    lam = A^-1 g,
    dL/dd_nu   = 2 N^-1 (d_nu - P_nu x) + N^-1 P_nu lam      (b depends on d)
    dL/dq_nu,k = -2 x_k . [B Y^T N^-1 (d - P x)]_nu           (explicit, chi^2)
                 + lam_k . [B Y^T N^-1 d]_nu                   (through b)
                 - lam_k . [B Y^T N^-1 P x]_nu - x_k . [B Y^T N^-1 P lam]_nu   (through A)

where [v]_nu . w_k means the inner product of the band-nu harmonic vector
v with component k's vector w over the modes both carry.  Spectral indices
enter through q_{nu,k}(beta); dq/dbeta follows from the SED (below).
"""
import math

import numpy as np

from . import sht

H_OVER_K = 0.04799243  # h / k_B in K / GHz


def sed_value(kind, freq, beta, nu_ref, temp=20.0):
    """Mixing scalar: 1 (CMB), (nu/nu_ref)^beta (power law), or the modified
    black body in Rayleigh-Jeans units (nu/nu_ref)^(beta+1) (e^x_ref - 1)/(e^x - 1)."""
    if kind == "cmb":
        return 1.0
    if kind == "sync":
        return (freq / nu_ref) ** beta
    x = H_OVER_K * freq / temp
    x0 = H_OVER_K * nu_ref / temp
    return (freq / nu_ref) ** (beta + 1.0) * math.expm1(x0) / math.expm1(x)


def sed_dbeta(kind, freq, beta, nu_ref, temp=20.0):
    """d q / d beta: both families are (nu/nu_ref)^beta times a beta-free factor."""
    if kind == "cmb":
        return 0.0
    return sed_value(kind, freq, beta, nu_ref, temp) * math.log(freq / nu_ref)


def band_dot(model, nu, v_band, k, w_comp):
    """[v]_nu . w_k over the modes band nu and component k share."""
    Lb = model.bands[nu]["lmax"]
    Lk = model.comps[k]["lmax"]
    L = min(Lb, Lk)
    return float(np.dot(sht.repack(v_band, Lb, L), sht.repack(w_comp, Lk, L)))


def band_adjoint(model, nu, f):
    """B_nu Y_nu^T f: band-nu harmonic vector of a pixel map (no mixing)."""
    b = model.bands[nu]
    ell = sht.lm_arrays(b["lmax"])[0]
    return b["beam"][ell] * sht.adjoint(b["grid"], b["lmax"], f)


def wf_loss_and_gradient(model, d, solve):
    """Loss, dL/dd (list of maps) and dL/dq [nbands, ncomp] at the Wiener
    filter x = A^-1 b.  solve(rhs) must return A^-1 rhs."""
    nb, nc = len(model.bands), len(model.comps)
    b = np.zeros(model.n)
    for nu, band in enumerate(model.bands):
        b = b + model.project_t(band["tau"] * d[nu], nu)
    x = solve(b)
    Sx = model.apply_prior_inv(x)
    resid = [d[nu] - model.project(x, nu) for nu in range(nb)]
    loss = 0.5 * float(x @ Sx) + sum(float(r @ (band["tau"] * r))
                                     for r, band in zip(resid, model.bands))
    g = Sx.copy()
    for nu, band in enumerate(model.bands):
        g = g - 2.0 * model.project_t(band["tau"] * resid[nu], nu)
    lam = solve(g)
    grad_d = []
    for nu, band in enumerate(model.bands):
        grad_d.append(2.0 * band["tau"] * resid[nu] + band["tau"] * model.project(lam, nu))
    xs, ls = model.split(x), model.split(lam)
    grad_q = np.zeros((nb, nc))
    for nu, band in enumerate(model.bands):
        tau = band["tau"]
        v_res = band_adjoint(model, nu, tau * resid[nu])
        v_d = band_adjoint(model, nu, tau * d[nu])
        v_px = band_adjoint(model, nu, tau * model.project(x, nu))
        v_pl = band_adjoint(model, nu, tau * model.project(lam, nu))
        for k in range(nc):
            grad_q[nu, k] = (-2.0 * band_dot(model, nu, v_res, k, xs[k])
                             + band_dot(model, nu, v_d, k, ls[k])
                             - band_dot(model, nu, v_px, k, ls[k])
                             - band_dot(model, nu, v_pl, k, xs[k]))
    return loss, grad_d, grad_q, x
