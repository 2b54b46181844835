"""Preconditioners (oracle).  TEST INFRASTRUCTURE ONLY.

Pseudo-inverse preconditioner, Sect. 3.3:
  * alpha_nu from App. A.1, eq:optimal-alpha:
        alpha^2 = sum_i t_i^2 / sum_i t_i,   t_i = tau_i / w_i
    (masked pixels, tau = 0, drop out of both sums).
  * A = U^T T U (eq:A-for-pseudoinv) with, per multipole l, the block
        U_l = [ alpha_nu b_{nu,l} q_{nu,k}  (band rows, eq:U-data)
                C_{k,l}^{-1/2} delta_{kk'}  (prior rows, eq:U-prior) ]
    restricted to bands with l <= L_nu and components with l <= L_k
    (zero padding elsewhere, end of Sect. 3.3).
  * U^+ = Moore-Penrose pseudo-inverse of U_l (Sect. 3.1), here by SVD.
  * M_PI = U^+ T^+ (U^+)^T (eq:fullmodel-preconditioner) with
        T^+ = blockdiag( alpha_nu^2 Y_nu^T W N_nu W Y_nu ,  I ).
    N_nu = diag(1/tau) is read as the pseudo-inverse of diag(tau): entries
    with tau = 0 (mask) are 0.
Observation merging (App. A.3): bands whose rows of U are (nearly)
proportional and whose normalised inverse-noise operators agree can share
one row in the preconditioner.  Each merge group keeps its first band (the
representative) with the row scaled by sqrt(1 + sum_nu gamma_{nu,l}^2),
gamma_{nu,l} the least-squares scale of band nu's row onto the
representative's at multipole l (the printed factor (gamma + 1)^{1/2} is read
as (1 + gamma^2)^{1/2}, the value for which the merged normal equations equal
the unmerged ones); the other bands of the group drop out of U^+ and T^+, so
T^+ needs the representative's SHTs only.  When the rows are exactly
proportional and the normalised noise operators equal, M_PI is unchanged.
Block-diagonal preconditioner, Sect. 5:
    M_diag = (U^T diag(T) U)^-1, one N_comp x N_comp block per (l, m, part);
    the alpha factors cancel, leaving
        D = sum_nu b_{nu,l}^2 diag(Y_nu^T N_nu^-1 Y_nu) q_nu q_nu^T + diag(C_{k,l}^-1),
    where diag(Y^T tau Y) at (l, m, part) = c_m^2 sum_r lambda_lm(z_r)^2
    sum_j tau_rj trig^2(m phi_rj)   (trig = cos for part 0, sin for part 1).
"""
import math

import numpy as np

from . import sht
from .legendre import LegendreSweep


def alpha_squared(tau, w):
    """eq:optimal-alpha (squared)."""
    t = np.asarray(tau, dtype=np.float64) / np.asarray(w, dtype=np.float64)
    s1 = t.sum()
    if s1 <= 0.0:
        raise ValueError("band has no unmasked pixel (sum tau/w = 0)")
    return float((t * t).sum() / s1)


def optimal_q(qmap):
    """App. A.2, eq:optimal-q: the scalar closest to a mixing map,
    sum_i q_i^2 / sum_i q_i over the map's pixels."""
    q = np.asarray(qmap, dtype=np.float64)
    return float((q * q).sum() / q.sum())


def effective_q(model):
    """Mixing scalars of the preconditioners: q_{nu,k}, or eq:optimal-q of the
    pair's mixing map where the mixing is spatially varying."""
    q = model.q.copy()
    for (nu, k), (_, qmap) in getattr(model, "mixing_maps", {}).items():
        q[nu, k] = optimal_q(qmap)
    return q


def u_blocks(model, alpha2):
    """U_l for l = 0..Lmax as an array [Lmax+1, nbands + ncomp, ncomp]."""
    nb, nc = len(model.bands), len(model.comps)
    lmax = max(max(b["lmax"] for b in model.bands), max(c["lmax"] for c in model.comps))
    U = np.zeros((lmax + 1, nb + nc, nc))
    alpha = np.sqrt(np.asarray(alpha2, dtype=np.float64))
    q = effective_q(model)
    for l in range(lmax + 1):
        for k, c in enumerate(model.comps):
            if l > c["lmax"]:
                continue
            for nu, b in enumerate(model.bands):
                if l <= b["lmax"]:
                    U[l, nu, k] = alpha[nu] * b["beam"][l] * q[nu, k]
            U[l, nb + k, k] = math.sqrt(c["invcl"][l])
    return U


def merge_rows(U, nb, merge):
    """Merged band rows of U (App. A.3): per group, the representative's row
    scaled by sqrt(1 + sum gamma_{nu,l}^2) and the other rows zeroed."""
    U = U.copy()
    for grp in merge or []:
        rep = grp[0]
        for l in range(U.shape[0]):
            u0 = U[l, rep]
            n0 = float(u0 @ u0)
            if n0 == 0.0:
                continue
            g2 = 0.0
            for nu in grp[1:]:
                g = float(U[l, nu] @ u0) / n0
                g2 += g * g
                U[l, nu] = 0.0
            U[l, rep] = math.sqrt(1.0 + g2) * u0
    return U


def u_pinv(model, alpha2, merge=None):
    """U_l^+ for every l, as [Lmax+1, ncomp, nbands + ncomp].

    Inactive columns (l > L_k) are dropped before the pseudo-inverse and
    come back as zero rows; all-zero rows of U_l give zero columns."""
    U = merge_rows(u_blocks(model, alpha2), len(model.bands), merge)
    nc = len(model.comps)
    lmax = U.shape[0] - 1
    P = np.zeros((lmax + 1, nc, U.shape[1]))
    for l in range(lmax + 1):
        act = [k for k, c in enumerate(model.comps) if l <= c["lmax"]]
        if not act:
            continue
        P[l][np.ix_(act, range(U.shape[1]))] = np.linalg.pinv(U[l][:, act])
    return P


class PseudoInversePrecond:
    """M_PI of eq:fullmodel-preconditioner (merge: optional list of band
    groups merged as in App. A.3)."""

    def __init__(self, model, merge=None):
        self.model = model
        nb = len(model.bands)
        self.alpha2 = np.array([alpha_squared(b["tau"], b["grid"].pixel_weights())
                                for b in model.bands])
        self.upinv = u_pinv(model, self.alpha2, merge)
        self.dropped = set(nu for grp in (merge or []) for nu in grp[1:])
        # T^+ pixel weight: alpha^2 W N W = alpha^2 w^2 tau^+
        self.tplus_w = []
        for nu, b in enumerate(model.bands):
            tau = np.asarray(b["tau"], dtype=np.float64)
            tinv = np.zeros_like(tau)
            pos = tau > 0
            tinv[pos] = 1.0 / tau[pos]
            w = b["grid"].pixel_weights()
            self.tplus_w.append(self.alpha2[nu] * w * w * tinv)
        self._ell_comp = [sht.lm_arrays(c["lmax"])[0] for c in model.comps]
        self._ell_band = [sht.lm_arrays(b["lmax"])[0] for b in model.bands]
        self.nb = nb

    def apply_ut(self, r):
        """(U^+)^T r: band parts t_nu (band layouts) and prior parts t_pr,k."""
        mdl = self.model
        rk = mdl.split(r)
        tb = []
        for nu, b in enumerate(mdl.bands):
            L = b["lmax"]
            acc = np.zeros(sht.nalm(L))
            for k, c in enumerate(mdl.comps):
                coef = self.upinv[self._ell_comp[k], k, nu]
                acc += sht.repack(coef * rk[k], c["lmax"], L)
            tb.append(acc)
        tp = []
        for kp, cp in enumerate(mdl.comps):
            acc = np.zeros(sht.nalm(cp["lmax"]))
            for k, c in enumerate(mdl.comps):
                coef = self.upinv[self._ell_comp[k], k, self.nb + kp]
                acc += sht.repack(coef * rk[k], c["lmax"], cp["lmax"])
            tp.append(acc)
        return tb, tp

    def apply_u(self, tb, tp):
        """U^+ applied to (band parts, prior parts)."""
        mdl = self.model
        out = []
        for k, c in enumerate(mdl.comps):
            acc = np.zeros(sht.nalm(c["lmax"]))
            for nu, b in enumerate(mdl.bands):
                coef = self.upinv[self._ell_band[nu], k, nu]
                acc += sht.repack(coef * tb[nu], b["lmax"], c["lmax"])
            for kp, cp in enumerate(mdl.comps):
                coef = self.upinv[self._ell_comp[kp], k, self.nb + kp]
                acc += sht.repack(coef * tp[kp], cp["lmax"], c["lmax"])
            out.append(acc)
        return mdl.join(out)

    def apply_tplus_band(self, t, nu):
        b = self.model.bands[nu]
        return sht.adjoint(b["grid"], b["lmax"],
                           self.tplus_w[nu] * sht.synth(b["grid"], b["lmax"], t))

    def __call__(self, r):
        tb, tp = self.apply_ut(r)
        tb = [np.zeros_like(t) if nu in self.dropped else self.apply_tplus_band(t, nu)
              for nu, t in enumerate(tb)]
        return self.apply_u(tb, tp)


def diag_yt_tau_y(grid, lmax, tau):
    """Diagonal of Y^T diag(tau) Y in the packed layout (plain definition
    evaluated ring by ring; the phi sums are direct)."""
    tau = np.asarray(tau, dtype=np.float64)
    ms = np.arange(lmax + 1)
    Gc = np.zeros((grid.nring, lmax + 1))
    Gs = np.zeros((grid.nring, lmax + 1))
    for r in range(grid.nring):
        o, n = grid.offset[r], grid.nphi[r]
        arg = np.outer(grid.ring_phi(r), ms)
        t = tau[o:o + n]
        Gc[r] = t @ (np.cos(arg) ** 2)
        Gs[r] = t @ (np.sin(arg) ** 2)
    out = np.zeros(sht.nalm(lmax))
    sweep = LegendreSweep(grid.z, grid.sint, lmax)
    for m in range(lmax + 1):
        lam2 = sweep.table(m) ** 2
        n = lmax - m + 1
        if m == 0:
            out[0:n] = Gc[:, 0] @ lam2
        else:
            o = sht.m_offset(lmax, m)
            out[o:o + n] = 2.0 * (Gc[:, m] @ lam2)
            out[o + n:o + 2 * n] = 2.0 * (Gs[:, m] @ lam2)
    return out


class DiagonalPrecond:
    """M_diag = (U^T diag(T) U)^-1 (Sect. 5), block inverse per coefficient."""

    def __init__(self, model):
        self.model = model
        nc = len(model.comps)
        self.lu = max(c["lmax"] for c in model.comps)
        ell_u, _, _ = sht.lm_arrays(self.lu)
        nu_ = sht.nalm(self.lu)
        D = np.zeros((nu_, nc, nc))
        for nu, b in enumerate(model.bands):
            dg = diag_yt_tau_y(b["grid"], b["lmax"], b["tau"])
            ell_b = sht.lm_arrays(b["lmax"])[0]
            dg = dg * b["beam"][ell_b] ** 2
            dg = sht.repack(dg, b["lmax"], self.lu)
            qe = effective_q(model)[nu]
            qq = np.outer(qe, qe)
            D += dg[:, None, None] * qq[None, :, :]
        active = np.zeros((nu_, nc))
        for k, c in enumerate(model.comps):
            act = ell_u <= c["lmax"]
            active[:, k] = act
            ic = np.zeros(nu_)
            ic[act] = c["invcl"][ell_u[act]]
            D[:, k, k] += ic
        D *= active[:, :, None] * active[:, None, :]
        for k in range(nc):
            D[:, k, k] += 1.0 - active[:, k]
        self.Dinv = np.linalg.inv(D)
        self.Dinv *= active[:, :, None] * active[:, None, :]

    def __call__(self, r):
        mdl = self.model
        ru = np.stack([sht.repack(rk, c["lmax"], self.lu)
                       for rk, c in zip(mdl.split(r), mdl.comps)], axis=1)
        zu = np.einsum("ikj,ij->ik", self.Dinv, ru)
        return mdl.join([sht.repack(zu[:, k], self.lu, c["lmax"])
                         for k, c in enumerate(mdl.comps)])
