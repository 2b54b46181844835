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


def test_power_law_sed_closed_forms():
    """(nu / nu_ref)^beta: 1 at the reference frequency, exact powers of two
    at octaves."""
    assert gradient.sed_value("sync", 30.0, -3.0, 30.0) == 1.0
    assert gradient.sed_value("sync", 60.0, -3.0, 30.0) == 0.125
    assert gradient.sed_value("sync", 15.0, -3.0, 30.0) == 8.0
    assert gradient.sed_value("cmb", 857.0, 0.0, 1.0) == 1.0


def _mbb_rj_planck(freq_ghz, beta, nu_ref_ghz, temp):
    """Modified black body nu^beta B_nu(T) converted to Rayleigh-Jeans
    brightness temperature (T_RJ = c^2 I / (2 k nu^2)), normalised at nu_ref,
    from the Planck function in SI units with the exact SI values of h and k
    (a different route to the same quantity as sed_value)."""
    import mpmath as mp
    h = mp.mpf("6.62607015e-34")
    k = mp.mpf("1.380649e-23")

    def t_rj(nu_hz):
        planck = nu_hz ** 3 / (mp.exp(h * nu_hz / (k * temp)) - 1)  # 2 h / c^2 cancels
        return nu_hz ** beta * planck / nu_hz ** 2
    return t_rj(mp.mpf(freq_ghz) * 10 ** 9) / t_rj(mp.mpf(nu_ref_ghz) * 10 ** 9)


def test_dust_sed_matches_planck_function():
    """The dust mixing scalar against the Planck-function definition (h / k in
    the oracle is the SI ratio rounded to 7 digits: relative agreement 1e-7).
    A wrong reference frequency, exponent (beta vs beta + 1) or h / k scale
    fails this."""
    import mpmath as mp
    for f in (30.0, 44.0, 143.0, 353.0, 545.0, 857.0):
        for beta, temp in ((1.6, 20.0), (1.2, 15.0), (2.0, 25.0)):
            with mp.workdps(40):
                ref = float(_mbb_rj_planck(f, beta, 353.0, temp))
            got = gradient.sed_value("dust", f, beta, 353.0, temp)
            assert abs(got - ref) <= 1e-7 * abs(ref), (f, beta, temp, got, ref)
    assert gradient.sed_value("dust", 353.0, 1.6, 353.0) == 1.0


def test_sed_beta_derivative_matches_high_precision_derivative():
    """d q / d beta against a 40-digit numerical derivative of the Planck-
    function form (mpmath), independent of sed_dbeta's closed form."""
    import mpmath as mp
    for f in (30.0, 100.0, 353.0, 857.0):
        for beta in (1.6, 1.3):
            with mp.workdps(40):
                ref = float(mp.diff(lambda b: _mbb_rj_planck(f, b, 353.0, 20.0), mp.mpf(beta)))
            got = gradient.sed_dbeta("dust", f, beta, 353.0, 20.0)
            assert abs(got - ref) <= 1e-7 * max(abs(ref), 1e-12), (f, beta, got, ref)
        for beta in (-3.0, -2.5):
            with mp.workdps(40):
                ref = float(mp.diff(lambda b: (mp.mpf(f) / 30) ** b, mp.mpf(beta)))
            got = gradient.sed_dbeta("sync", f, beta, 30.0)
            assert abs(got - ref) <= 1e-13 * max(abs(ref), 1e-12), (f, beta, got, ref)


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
