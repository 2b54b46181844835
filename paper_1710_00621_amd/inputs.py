"""Seeded synthetic inputs for the solver (shared by tests and benchmarks).

This module only *describes and draws inputs*: band/component layouts,
beam transfer functions, prior spectra, mixing scalars, noise RMS maps,
masks and random signal vectors.  It holds none of the solver's arithmetic
(no transform, no operator, no preconditioner), so both the HIP library and
the CPU oracle can be fed from it without sharing any of their code.

Workload recipes (the paper's Planck-derived inputs are not available; these
keep its structure: several bands with different resolutions and Gaussian
beams, inhomogeneous noise, masks, and a prior crossing the noise at mid-l,
Sect. 5):

  tiny      1 comp (CMB), 1 band on a Gauss-Legendre grid of 33 x 65,
            L = 32, beam FWHM 10 deg, noise RMS ~ U[0.5, 1.5].
  multires  CMB + power law (beta = -3, 30 GHz), bands 30/70/100/143/217 GHz
            at Nside 64/128/128/256/256, L_nu = 2 Nside, FWHM 60/30/20/10/7',
            L_k = 512, RMS = exp(0.3 z), full sky.
  masked    CMB + synchrotron (beta = -3) + dust (beta = 1.6, T = 20 K,
            353 GHz), 9 bands 30..857 GHz at Nside 512 (x3) / 1024 (x6),
            L_nu = min(2000, 2 Nside), FWHM 30 (1/6)^(i/8) arcmin, L_k = 2000,
            RMS = exp(0.3 z), mask |b| < 15 deg plus 500 disks of 1 deg.
  batched   64 problems shaped like multires with Nside_max in {64,128,256},
            1-3 components, sky fraction ~ U[0.6, 0.95].
  diff      7 bands 30..353 GHz at Nside 256, L = 512, FWHM 37.5', RMS ~
            U[0.5, 1.5], CMB + synchrotron + dust, full sky.
  fullres   the masked recipe's 9 bands and components at full Planck-like
            resolution: Nside 1024 (x3) / 2048 (x6), L_nu = min(6000, 2
            Nside), L_k = 6000, full sky, Wiener filter.
Every recipe also has a ``scale`` knob that divides Nside and every
band-limit (and multiplies the FWHM) to give small copies for the oracle.

Priors: CMB C_l = 1/(l(l+1)) for l >= 2 (no prior below); foregrounds
C_l = 10 l^-2.5 for l >= 1 (no prior at l = 0).  C^-1 = 0 means no prior.
Mixing: CMB 1; power law (nu/nu_ref)^beta; dust modified black body in
Rayleigh-Jeans units (nu/353)^(beta+1) (e^x353 - 1)/(e^x - 1), x = h nu/(k T).
"""
import math

import numpy as np

H_OVER_K_GHZ = 0.04799243  # h / k_B in K / GHz


# --------------------------------------------------------------------------
# tables that define a model
# --------------------------------------------------------------------------
def gaussian_beam(fwhm_arcmin, lmax):
    """b_l = exp(-l(l+1) sigma^2 / 2), sigma = FWHM / sqrt(8 ln 2) (radians)."""
    sig = fwhm_arcmin / 60.0 * math.pi / 180.0 / math.sqrt(8.0 * math.log(2.0))
    l = np.arange(lmax + 1, dtype=np.float64)
    return np.exp(-0.5 * l * (l + 1.0) * sig * sig)


def inv_cl(kind, lmax, amplitude=1.0):
    """C_l^-1 tables; 0 where the component has no prior."""
    l = np.arange(lmax + 1, dtype=np.float64)
    out = np.zeros(lmax + 1)
    if kind == "cmb":
        out[2:] = l[2:] * (l[2:] + 1.0) / amplitude
    elif kind == "powerlaw":
        out[1:] = l[1:] ** 2.5 / (10.0 * amplitude)
    elif kind == "none":
        pass
    else:
        raise ValueError(kind)
    return out


def sed(comp, freq_ghz):
    """Mixing scalar q_{nu,k} for a spatially constant SED."""
    kind = comp["kind"]
    if kind == "cmb":
        return 1.0
    if kind == "sync":
        return (freq_ghz / comp.get("nu_ref", 30.0)) ** comp["beta"]
    if kind == "dust":
        nu0 = comp.get("nu_ref", 353.0)
        T = comp.get("T", 20.0)
        x = H_OVER_K_GHZ * freq_ghz / T
        x0 = H_OVER_K_GHZ * nu0 / T
        return (freq_ghz / nu0) ** (comp["beta"] + 1.0) * math.expm1(x0) / math.expm1(x)
    raise ValueError(kind)


def sed_dlogbeta(comp, freq_ghz):
    """d q / d beta = q ln(nu / nu_ref) for both SED families."""
    if comp["kind"] == "cmb":
        return 0.0
    return sed(comp, freq_ghz) * math.log(freq_ghz / comp.get(
        "nu_ref", 30.0 if comp["kind"] == "sync" else 353.0))


def grid_npix(spec):
    if spec[0] == "healpix":
        return 12 * spec[1] * spec[1]
    if spec[0] == "gl":
        return spec[1] * spec[2]
    raise ValueError(spec)


def grid_nring(spec):
    if spec[0] == "healpix":
        return 4 * spec[1] - 1
    return spec[1]


CMB = {"kind": "cmb", "prior": "cmb"}
SYNC = {"kind": "sync", "beta": -3.0, "nu_ref": 30.0, "prior": "powerlaw"}
DUST = {"kind": "dust", "beta": 1.6, "T": 20.0, "nu_ref": 353.0, "prior": "powerlaw"}


def _problem(bands, comps, noise, mask, seed, name, rhs="wf"):
    q = np.array([[sed(c, b["freq"]) for c in comps] for b in bands])
    return {"name": name, "bands": bands, "comps": comps, "q": q,
            "noise": noise, "mask": mask, "seed": seed, "rhs": rhs}


def make_problem(name, scale=1, index=0):
    """Describe one workload (see the module docstring).  ``scale`` divides
    Nside and every band-limit; ``index`` picks one problem of ``batched``."""
    s = int(scale)
    if name == "tiny":
        L = 32 // s if s > 1 else 32
        bands = [{"freq": 143.0, "grid": ("gl", L + 1, 2 * L + 1), "lmax": L,
                  "fwhm": 600.0 * s}]
        comps = [dict(CMB, lmax=L)]
        return _problem(bands, comps, ("uniform", 0.5, 1.5), None, 1, name)
    if name == "multires":
        ns = [64, 128, 128, 256, 256]
        fw = [60.0, 30.0, 20.0, 10.0, 7.0]
        fr = [30.0, 70.0, 100.0, 143.0, 217.0]
        bands = [{"freq": f, "grid": ("healpix", n // s), "lmax": 2 * (n // s),
                  "fwhm": w * s} for f, n, w in zip(fr, ns, fw)]
        comps = [dict(CMB, lmax=512 // s), dict(SYNC, lmax=512 // s)]
        return _problem(bands, comps, ("lognormal", 0.3), None, 2, name)
    if name == "masked":
        fr = [30.0, 44.0, 70.0, 100.0, 143.0, 217.0, 353.0, 545.0, 857.0]
        bands = []
        for i, f in enumerate(fr):
            n = (512 if i < 3 else 1024) // s
            bands.append({"freq": f, "grid": ("healpix", n),
                          "lmax": min(2000 // s, 2 * n),
                          "fwhm": 30.0 * (1.0 / 6.0) ** (i / 8.0) * s})
        comps = [dict(CMB, lmax=2000 // s), dict(SYNC, lmax=2000 // s),
                 dict(DUST, lmax=2000 // s)]
        return _problem(bands, comps, ("lognormal", 0.3),
                        ("galactic_disks", math.sin(math.radians(15.0)), 500), 3, name,
                        rhs="cr")
    if name == "fullres":
        fr = [30.0, 44.0, 70.0, 100.0, 143.0, 217.0, 353.0, 545.0, 857.0]
        bands = []
        for i, f in enumerate(fr):
            n = (1024 if i < 3 else 2048) // s
            bands.append({"freq": f, "grid": ("healpix", n),
                          "lmax": min(6000 // s, 2 * n),
                          "fwhm": 30.0 * (1.0 / 6.0) ** (i / 8.0) * s})
        comps = [dict(CMB, lmax=6000 // s), dict(SYNC, lmax=6000 // s),
                 dict(DUST, lmax=6000 // s)]
        return _problem(bands, comps, ("lognormal", 0.3), None, 6, name)
    if name == "batched":
        i = int(index)
        nmax_full = (64, 128, 256)[i % 3]
        nmax = nmax_full // s
        fr = [30.0, 70.0, 100.0, 143.0, 217.0]
        fw = [60.0, 30.0, 20.0, 10.0, 7.0]
        fac = (0.25, 0.5, 0.5, 1.0, 1.0)
        bands = [{"freq": f, "grid": ("healpix", max(1, int(nmax * a))),
                  "lmax": 2 * max(1, int(nmax * a)),
                  "fwhm": w * 256.0 / nmax_full * s}
                 for f, w, a in zip(fr, fw, fac)]
        ncomp = 1 + (i // 3) % 3
        comps = [dict(c, lmax=2 * nmax) for c in (CMB, SYNC, DUST)[:ncomp]]
        rng = np.random.default_rng(400 + i)
        fsky = float(rng.uniform(0.6, 0.95))
        return _problem(bands, comps, ("lognormal", 0.3),
                        ("fsky", fsky), 400 + i, name, rhs="cr")
    if name == "diff":
        fr = [30.0, 44.0, 70.0, 100.0, 143.0, 217.0, 353.0]
        n = 256 // s
        bands = [{"freq": f, "grid": ("healpix", n), "lmax": 2 * n,
                  "fwhm": 37.5 * s} for f in fr]
        comps = [dict(c, lmax=2 * n) for c in (CMB, SYNC, DUST)]
        return _problem(bands, comps, ("uniform", 0.5, 1.5), None, 5, name)
    raise ValueError(f"unknown workload {name!r}")


def beams(problem):
    return [gaussian_beam(b["fwhm"], b["lmax"]) for b in problem["bands"]]


def priors(problem):
    return [inv_cl(c["prior"], c["lmax"]) for c in problem["comps"]]


# --------------------------------------------------------------------------
# random draws
# --------------------------------------------------------------------------
def _disk_mask(z, phi, centres_z, centres_phi, radius_rad, masked, target=None,
               order=None):
    """Mask pixels within radius of each centre; stop early at ``target``."""
    cr = math.cos(radius_rad)
    st = np.sqrt(np.maximum(0.0, (1.0 - z) * (1.0 + z)))
    if order is None:
        order = np.argsort(z, kind="stable")
    zs = z[order]
    npix = len(z)
    nmask = int(masked.sum())
    for zc, pc in zip(centres_z, centres_phi):
        thc = math.acos(max(-1.0, min(1.0, zc)))
        zlo = math.cos(min(math.pi, thc + radius_rad))
        zhi = math.cos(max(0.0, thc - radius_rad))
        i0 = np.searchsorted(zs, zlo, side="left")
        i1 = np.searchsorted(zs, zhi, side="right")
        idx = order[i0:i1]
        sc = math.sqrt(max(0.0, (1.0 - zc) * (1.0 + zc)))
        cosd = z[idx] * zc + st[idx] * sc * np.cos(phi[idx] - pc)
        hit = idx[(cosd >= cr) & ~masked[idx]]
        masked[hit] = True
        nmask += len(hit)
        if target is not None and nmask >= target * npix:
            break
    return masked


def make_mask(mask_spec, z, phi, seed):
    """Boolean mask (True = masked) for the given pixel centres."""
    if mask_spec is None:
        return np.zeros(len(z), dtype=bool)
    rng = np.random.default_rng([seed, 77])
    if mask_spec[0] == "galactic_disks":
        _, sin_cut, ndisk = mask_spec
        masked = np.abs(z) < sin_cut
        cz = rng.uniform(-1.0, 1.0, ndisk)
        cp = rng.uniform(0.0, 2.0 * math.pi, ndisk)
        return _disk_mask(z, phi, cz, cp, math.radians(1.0), masked)
    if mask_spec[0] == "fsky":
        fsky = mask_spec[1]
        masked = np.abs(z) < 0.5 * (1.0 - fsky)
        order = np.argsort(z, kind="stable")
        while masked.mean() < 1.0 - fsky:
            cz = rng.uniform(-1.0, 1.0, 64)
            cp = rng.uniform(0.0, 2.0 * math.pi, 64)
            masked = _disk_mask(z, phi, cz, cp, math.radians(1.0), masked,
                                target=1.0 - fsky, order=order)
        return masked
    raise ValueError(mask_spec)


def noise_rms(problem, band_index, npix):
    """Per-pixel noise RMS of one band."""
    rng = np.random.default_rng([problem["seed"], 11, band_index])
    kind = problem["noise"]
    if kind[0] == "uniform":
        return rng.uniform(kind[1], kind[2], npix)
    if kind[0] == "lognormal":
        return np.exp(kind[1] * rng.standard_normal(npix))
    raise ValueError(kind)


def inverse_noise_maps(problem, centres):
    """tau_nu = sigma^-2 per band, 0 inside the mask.

    ``centres(grid_spec) -> (z, phi)`` supplies the pixel centres (in ring
    order) of a grid; it is needed only when the recipe has a mask."""
    taus = []
    cache = {}
    for nu, b in enumerate(problem["bands"]):
        npix = grid_npix(b["grid"])
        sig = noise_rms(problem, nu, npix)
        tau = 1.0 / (sig * sig)
        if problem["mask"] is not None:
            key = b["grid"]
            if key not in cache:
                z, phi = centres(b["grid"])
                cache[key] = make_mask(problem["mask"], np.asarray(z), np.asarray(phi),
                                       problem["seed"])
            tau = np.where(cache[key], 0.0, tau)
        taus.append(tau)
    return taus


def signal_coefficients(problem, rhs=0):
    """s_k ~ N(0, C_k) per real coefficient (0 where there is no prior),
    concatenated over components in the packed m-major layout.  The variance
    depends only on l, so the per-coefficient l is needed: it is recomputed
    here from the layout (m = 0: l = 0..L; m >= 1: cosine then sine blocks)."""
    rng = np.random.default_rng([problem["seed"], 23, rhs])
    out = []
    for c, icl in zip(problem["comps"], priors(problem)):
        L = c["lmax"]
        ell = _packed_ell(L)
        cl = np.zeros(L + 1)
        pos = icl > 0
        cl[pos] = 1.0 / icl[pos]
        out.append(np.sqrt(cl[ell]) * rng.standard_normal(len(ell)))
    return np.concatenate(out)


def _packed_ell(L):
    parts = [np.arange(L + 1)]
    for m in range(1, L + 1):
        blk = np.arange(m, L + 1)
        parts.append(blk)
        parts.append(blk)
    return np.concatenate(parts)


def white_noise(problem, band_index, npix, rhs=0):
    """Standard normal noise realisation z for d = P s + sigma z."""
    rng = np.random.default_rng([problem["seed"], 31, band_index, rhs])
    return rng.standard_normal(npix)


def random_vector(n, seed):
    return np.random.default_rng([seed, 47]).standard_normal(n)
