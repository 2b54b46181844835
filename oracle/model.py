"""The constrained-realization linear system (oracle).  TEST INFRASTRUCTURE ONLY.

Sect. 2.2: components s_k (harmonic, band-limit L_k) reach sky map d_nu
through P_{nu,k} = Y_nu B_nu Q~_{nu,k} (eq:P).  With spatially constant
mixing, Q~_{nu,k} = q_{nu,k} I (Sect. 3.3), B_nu is diagonal in harmonic
space with b_{nu,l}, and band nu carries harmonic modes up to L_nu.  The
noise is diagonal in pixel space, N_nu^-1 = diag(tau_nu) with tau = 0 in
masked pixels, and the prior S is diagonal in harmonic space with C_{k,l}
(C^-1 = 0 where a component has no prior).

Sect. 2.3, eq:A:  A = S^-1 + P^T N^-1 P.

Input arrays (all float64):
    bands: list of dict(grid=Grid, lmax=L_nu, beam=b[0..L_nu], tau=tau[npix])
    comps: list of dict(lmax=L_k, invcl=C^-1[0..L_k])
    q:     mixing matrix [nbands, ncomp]
A component vector x is the concatenation of the packed harmonic vectors
of all components (lengths (L_k+1)^2).
"""
import numpy as np

from . import sht


class Model:
    def __init__(self, bands, comps, q, mixing_maps=None):
        self.bands = bands
        self.comps = comps
        self.q = np.asarray(q, dtype=np.float64).reshape(len(bands), len(comps))
        # spatially varying mixing (eq:Q): {(nu, k): (grid, q map)}; the pair's
        # block of P is Y_nu B_nu Q~ with Q~ = Y^T W Q Y on that grid at L_k
        self.mixing_maps = dict(mixing_maps or {})
        self.sizes = [sht.nalm(c["lmax"]) for c in comps]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.n = int(self.offsets[-1])
        self._ell_band = [sht.lm_arrays(b["lmax"])[0] for b in bands]
        self._ell_comp = [sht.lm_arrays(c["lmax"])[0] for c in comps]

    # -- vector helpers -------------------------------------------------
    def split(self, x):
        x = np.asarray(x, dtype=np.float64)
        return [x[self.offsets[k]:self.offsets[k + 1]] for k in range(len(self.comps))]

    def join(self, parts):
        return np.concatenate(parts)

    # -- pieces of P (eq:P with Q~ = q I) --------------------------------
    def mix(self, nu, k, xk):
        """Q~_{nu,k} x_k (eq:Q): q_{nu,k} x_k for spatially constant mixing, else
        Y^T W (q map) Y x_k on the pair's grid, output at the component's L_k."""
        if (nu, k) not in self.mixing_maps:
            return self.q[nu, k] * xk
        grid, qmap = self.mixing_maps[(nu, k)]
        L = self.comps[k]["lmax"]
        f = sht.synth(grid, L, xk)
        return sht.adjoint(grid, L, grid.pixel_weights() * np.asarray(qmap) * f)

    def to_band(self, x, nu):
        """u_nu = B_nu sum_k Q~_{nu,k} x_k, in band nu's packed layout."""
        L = self.bands[nu]["lmax"]
        u = np.zeros(sht.nalm(L))
        for k, xk in enumerate(self.split(x)):
            u += sht.repack(self.mix(nu, k, xk), self.comps[k]["lmax"], L)
        return self.bands[nu]["beam"][self._ell_band[nu]] * u

    def from_band(self, v, nu):
        """Transpose of to_band: component vector from a band vector (Q~ is
        symmetric: W and Q are both diagonal)."""
        bv = self.bands[nu]["beam"][self._ell_band[nu]] * v
        parts = [self.mix(nu, k, sht.repack(bv, self.bands[nu]["lmax"], c["lmax"]))
                 for k, c in enumerate(self.comps)]
        return self.join(parts)

    def project(self, x, nu, ms=None):
        """P_nu x: pixel map of band nu (ms: only these m are synthesised, the
        other m of x taken as zero)."""
        b = self.bands[nu]
        return sht.synth(b["grid"], b["lmax"], self.to_band(x, nu), ms=ms)

    def project_t(self, f, nu, ms=None):
        """P_nu^T f for a pixel map f of band nu (ms: only these m computed)."""
        b = self.bands[nu]
        return self.from_band(sht.adjoint(b["grid"], b["lmax"], f, ms=ms), nu)

    def apply_prior_inv(self, x):
        """S^-1 x (diagonal, C_{k,l}^-1 per coefficient)."""
        parts = [c["invcl"][self._ell_comp[k]] * xk
                 for k, (c, xk) in enumerate(zip(self.comps, self.split(x)))]
        return self.join(parts)

    def apply_A(self, x, ms_in=None, ms_out=None):
        """A x = S^-1 x + sum_nu P_nu^T N_nu^-1 P_nu x (eq:A).

        ms_in / ms_out (optional, for sampled checks at large sizes): x is
        nonzero only at the m in ms_in, and only the outputs at the m in
        ms_out are wanted (the others are returned as zero)."""
        y = self.apply_prior_inv(x)
        if ms_out is not None:
            keep = np.zeros(self.n, dtype=bool)
            for k, c in enumerate(self.comps):
                mm = sht.lm_arrays(c["lmax"])[1]
                keep[self.offsets[k]:self.offsets[k + 1]] = np.isin(mm, list(ms_out))
            y = np.where(keep, y, 0.0)
        for nu, b in enumerate(self.bands):
            y = y + self.project_t(b["tau"] * self.project(x, nu, ms=ms_in), nu, ms=ms_out)
        return y
