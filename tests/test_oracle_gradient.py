"""Pins for the oracle's implicit gradients of the Wiener-filter loss:
central finite differences on a tiny model solved exactly (dense
Cholesky), the stationarity identity dL/dx = -S^-1 x at the Wiener filter,
and the SED derivative."""
import numpy as np
import scipy.linalg

from oracle import dense, geometry, gradient
from oracle.model import Model
from paper_1710_00621_amd import inputs

FREQS = [30.0, 70.0, 143.0, 353.0]
KINDS = [("cmb", None, None), ("sync", -3.0, 30.0), ("dust", 1.6, 353.0)]


def _model(beta, seed=3):
    rng = np.random.default_rng(seed)
    specs = [("healpix", 4), ("healpix", 4), ("healpix", 8), ("healpix", 8)]
    Ls = [8, 8, 12, 12]
    bands = []
    for spec, L, f in zip(specs, Ls, FREQS):
        g = geometry.make_grid(spec)
        tau = np.exp(0.4 * rng.standard_normal(g.npix)) * 4.0
        bands.append({"grid": g, "lmax": L, "beam": inputs.gaussian_beam(400.0, L), "tau": tau})
    comps = [{"lmax": 10, "invcl": inputs.inv_cl("cmb", 10, amplitude=0.05)},
             {"lmax": 10, "invcl": inputs.inv_cl("powerlaw", 10, amplitude=0.05)},
             {"lmax": 10, "invcl": inputs.inv_cl("powerlaw", 10, amplitude=0.05)}]
    q = np.array([[gradient.sed_value(kind, f, beta[j] if j else 0.0, ref or 1.0)
                   for j, (kind, _, ref) in enumerate(KINDS)] for f in FREQS])
    return Model(bands, comps, q)


def _data(mdl, seed=5):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(b["grid"].npix) for b in mdl.bands]


def _solver(mdl):
    cf = scipy.linalg.cho_factor(dense.dense_a(mdl))
    return lambda v: scipy.linalg.cho_solve(cf, v)


def _loss(beta, d):
    mdl = _model(beta)
    return gradient.wf_loss_and_gradient(mdl, d, _solver(mdl))


def test_sed_derivative_matches_finite_difference():
    for kind, beta, ref in KINDS[1:]:
        for f in FREQS:
            h = 1e-6
            fd = (gradient.sed_value(kind, f, beta + h, ref) - gradient.sed_value(kind, f, beta - h, ref)) / (2 * h)
            assert abs(gradient.sed_dbeta(kind, f, beta, ref) - fd) <= 1e-7 * max(1.0, abs(fd))


def test_stationarity_at_wiener_filter():
    """At x = A^-1 b the explicit gradient S^-1 x - 2 P^T N^-1 (d - P x)
    equals -S^-1 x (since A x = b)."""
    beta = [0.0, -3.0, 1.6]
    mdl = _model(beta)
    d = _data(mdl)
    solve = _solver(mdl)
    b = sum(mdl.project_t(bd["tau"] * d[nu], nu) for nu, bd in enumerate(mdl.bands))
    x = solve(b)
    Sx = mdl.apply_prior_inv(x)
    g = Sx.copy()
    for nu, bd in enumerate(mdl.bands):
        g -= 2.0 * mdl.project_t(bd["tau"] * (d[nu] - mdl.project(x, nu)), nu)
    np.testing.assert_allclose(g, -Sx, atol=1e-9 * np.abs(Sx).max())


def test_beta_gradient_matches_central_differences():
    beta = [0.0, -3.0, 1.6]
    d = _data(_model(beta))
    L0, gd, gq, _ = _loss(beta, d)
    for j in (1, 2):
        kind, _, ref = KINDS[j]
        analytic = sum(gq[nu, j] * gradient.sed_dbeta(kind, f, beta[j], ref) for nu, f in enumerate(FREQS))
        h = 1e-5
        bp, bm = list(beta), list(beta)
        bp[j] += h
        bm[j] -= h
        fd = (_loss(bp, d)[0] - _loss(bm, d)[0]) / (2 * h)
        assert abs(analytic - fd) <= 1e-6 * abs(fd), (j, analytic, fd)


def test_data_gradient_matches_central_differences():
    beta = [0.0, -3.0, 1.6]
    mdl = _model(beta)
    d = _data(mdl)
    solve = _solver(mdl)
    L0, gd, gq, _ = gradient.wf_loss_and_gradient(mdl, d, solve)
    rng = np.random.default_rng(9)
    for _ in range(3):
        dirs = [rng.standard_normal(len(v)) for v in d]
        h = 1e-4
        dp = [v + h * w for v, w in zip(d, dirs)]
        dm = [v - h * w for v, w in zip(d, dirs)]
        fd = (gradient.wf_loss_and_gradient(mdl, dp, solve)[0] -
              gradient.wf_loss_and_gradient(mdl, dm, solve)[0]) / (2 * h)
        analytic = sum(float(g @ w) for g, w in zip(gd, dirs))
        assert abs(analytic - fd) <= 1e-7 * abs(fd)


def test_mixing_gradient_matches_central_differences_in_q():
    """Each q_{nu,k} perturbed on its own (the model is linear in q inside P)."""
    beta = [0.0, -3.0, 1.6]
    mdl = _model(beta)
    d = _data(mdl)
    L0, gd, gq, _ = gradient.wf_loss_and_gradient(mdl, d, _solver(mdl))
    for nu, k in ((0, 0), (2, 1), (3, 2)):
        h = 1e-6
        vals = []
        for sgn in (1, -1):
            m2 = Model(mdl.bands, mdl.comps, mdl.q.copy())
            m2.q[nu, k] += sgn * h
            vals.append(gradient.wf_loss_and_gradient(m2, d, _solver(m2))[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(gq[nu, k] - fd) <= 1e-6 * max(abs(fd), 1e-3 * abs(L0)), (nu, k, gq[nu, k], fd)
