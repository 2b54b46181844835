"""Test helpers: build oracle models from the shared seeded input recipes."""
import numpy as np

from oracle import geometry, sht
from oracle.model import Model
from paper_1710_00621_amd import inputs


def grid_centres(spec):
    return geometry.make_grid(spec).pixel_centres()


def oracle_model(problem, taus=None):
    """Oracle Model + the tau maps used (tau from the recipe unless given)."""
    if taus is None:
        taus = inputs.inverse_noise_maps(problem, grid_centres)
    bl = inputs.beams(problem)
    bands = []
    for b, beam, tau in zip(problem["bands"], bl, taus):
        bands.append({"grid": geometry.make_grid(b["grid"]), "lmax": b["lmax"],
                      "beam": beam, "tau": np.asarray(tau, dtype=np.float64)})
    comps = [{"lmax": c["lmax"], "invcl": icl}
             for c, icl in zip(problem["comps"], inputs.priors(problem))]
    return Model(bands, comps, problem["q"]), taus


def synthetic_data(problem, model, rhs=0):
    """d_nu = P_nu s + sigma_nu z (oracle projection)."""
    s = inputs.signal_coefficients(problem, rhs)
    d = []
    for nu, b in enumerate(model.bands):
        npix = b["grid"].npix
        tau = b["tau"]
        sig = np.zeros(npix)
        pos = tau > 0
        sig[pos] = 1.0 / np.sqrt(tau[pos])
        d.append(model.project(s, nu) + sig * inputs.white_noise(problem, nu, npix, rhs))
    return s, d


def small_model(ncomp=2, seed=0, mask=False, grids=(("healpix", 4), ("healpix", 8)),
                lmax_bands=(8, 16), lmax_comps=(12, 16)):
    """A hand-made multi-resolution model for quick tests."""
    rng = np.random.default_rng(seed)
    bands = []
    for spec, L in zip(grids, lmax_bands):
        g = geometry.make_grid(spec)
        tau = np.exp(0.6 * rng.standard_normal(g.npix))
        if mask:
            z, _ = g.pixel_centres()
            tau[np.abs(z) < 0.2] = 0.0
        beam = inputs.gaussian_beam(300.0 * 8 / L, L)
        bands.append({"grid": g, "lmax": L, "beam": beam, "tau": tau})
    comps = []
    kinds = ["cmb", "powerlaw", "powerlaw"]
    for k in range(ncomp):
        L = lmax_comps[k % len(lmax_comps)]
        comps.append({"lmax": L, "invcl": inputs.inv_cl(kinds[k], L, amplitude=0.05)})
    q = np.abs(rng.normal(1.0, 0.5, (len(bands), ncomp))) + 0.2
    return Model(bands, comps, q)


def rel_max(a, b):
    """max |a - b| / max |b|: an element-wise comparison on the scale of b."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
