"""Pins for the oracle's linear system, preconditioners, PCG and RHS."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import dense, geometry, pcg, philox, precond, rhs, sht
from oracle.model import Model
from paper_1710_00621_amd import inputs
from tests.helpers import oracle_model, small_model, synthetic_data


def test_apply_a_matches_dense_and_is_spd():
    mdl = small_model(ncomp=2, mask=True)
    A = dense.dense_a(mdl)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(mdl.n)
    np.testing.assert_allclose(mdl.apply_A(x), A @ x, rtol=1e-11, atol=1e-11 * np.abs(A @ x).max())
    assert np.max(np.abs(A - A.T)) < 1e-11 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0


def test_alpha_closed_form():
    w = np.full(48, 4 * math.pi / 48)
    assert abs(precond.alpha_squared(3.7 * w, w) - 3.7) < 1e-14
    tau = np.array([1.0, 2.0, 0.0, 4.0])
    w = np.array([1.0, 1.0, 1.0, 2.0])
    # t = (1, 2, 0, 2): sum t^2 / sum t = 9 / 5
    assert abs(precond.alpha_squared(tau, w) - 9.0 / 5.0) < 1e-15


def test_u_pinv_is_left_inverse_and_normal_equations():
    """Sect. 3.1: for full column rank U^+ = (U^T U)^-1 U^T and U^+ U = I;
    otherwise U^+ is the Moore-Penrose inverse (Penrose conditions)."""
    mdl = small_model(ncomp=3)
    a2 = np.array([1.3, 0.7])
    U = precond.u_blocks(mdl, a2)
    P = precond.u_pinv(mdl, a2)
    nfull = 0
    for l in range(U.shape[0]):
        act = [k for k, c in enumerate(mdl.comps) if l <= c["lmax"]]
        Ua = U[l][:, act]
        Pa = P[l][act, :]
        tol = 1e-10 * max(1.0, np.abs(Pa).max() * np.abs(Ua).max())
        np.testing.assert_allclose(Ua @ Pa @ Ua, Ua, atol=tol * np.abs(Ua).max())
        np.testing.assert_allclose(Pa @ Ua @ Pa, Pa, atol=tol * np.abs(Pa).max())
        np.testing.assert_allclose(Ua @ Pa, (Ua @ Pa).T, atol=tol)
        np.testing.assert_allclose(Pa @ Ua, (Pa @ Ua).T, atol=tol)
        if np.linalg.matrix_rank(Ua) == len(act):
            nfull += 1
            np.testing.assert_allclose(Pa @ Ua, np.eye(len(act)), atol=1e-12)
            ref = np.linalg.solve(Ua.T @ Ua, Ua.T)
            np.testing.assert_allclose(Pa, ref, atol=1e-10 * np.abs(ref).max())
    assert nfull >= U.shape[0] - 2


def _gl_flat_model(ncomp=2):
    """GL bands with tau proportional to the quadrature weight: T = I exactly."""
    rng = np.random.default_rng(4)
    bands = []
    for L, t0 in ((12, 3.0), (16, 0.5), (10, 7.0)):
        g = geometry.gauss_legendre(L + 1, 2 * L + 1)
        bands.append({"grid": g, "lmax": L, "beam": inputs.gaussian_beam(400.0, L),
                      "tau": t0 * g.pixel_weights()})
    comps = [{"lmax": 16, "invcl": inputs.inv_cl("cmb", 16, 0.1)},
             {"lmax": 14, "invcl": inputs.inv_cl("powerlaw", 14, 0.1)}][:ncomp]
    q = np.abs(rng.normal(1.0, 0.4, (3, ncomp))) + 0.1
    return Model(bands, comps, q)


def test_pinv_preconditioner_exact_for_flat_noise():
    """Flat inverse noise (tau/w constant on an exact-quadrature grid) gives
    T = T^+ = I and M_PI A = I (Sect. 3.3, first special case)."""
    mdl = _gl_flat_model()
    M = precond.PseudoInversePrecond(mdl)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(mdl.n)
    np.testing.assert_allclose(M(mdl.apply_A(x)), x, atol=1e-11 * np.abs(x).max())
    b = mdl.apply_A(x)
    res = pcg.pcg(mdl.apply_A, M, b, rtol=1e-10, maxiter=10)
    assert res.status == "ok" and res.iters == 1


def test_diag_equals_pinv_for_flat_noise():
    """With T = I both preconditioners reduce to (U^T U)^-1 (Sect. 3.2 figure note)."""
    mdl = _gl_flat_model()
    Mp = precond.PseudoInversePrecond(mdl)
    Md = precond.DiagonalPrecond(mdl)
    x = np.random.default_rng(8).standard_normal(mdl.n)
    np.testing.assert_allclose(Md(x), Mp(x), atol=1e-11 * np.abs(Mp(x)).max())


def test_pinv_single_component_reduces_to_simplest():
    """1 component, 1 band, no prior: M_PI = B^-1 Y^T W N W Y B^-1
    (eq:simplest-preconditioner), built here from dense matrices."""
    g = geometry.healpix(4)
    L = 8
    rng = np.random.default_rng(6)
    tau = np.exp(0.5 * rng.standard_normal(g.npix))
    beam = inputs.gaussian_beam(500.0, L)
    mdl = Model([{"grid": g, "lmax": L, "beam": beam, "tau": tau}],
                [{"lmax": L, "invcl": np.zeros(L + 1)}], np.array([[1.0]]))
    M = precond.PseudoInversePrecond(mdl)
    Y = dense.dense_y(g, L)
    w = g.pixel_weights()
    binv = 1.0 / beam[sht.lm_arrays(L)[0]]
    Mref = binv[:, None] * (Y.T @ ((w * w / tau)[:, None] * Y)) * binv[None, :]
    x = rng.standard_normal(mdl.n)
    np.testing.assert_allclose(M(x), Mref @ x, rtol=1e-10, atol=1e-10 * np.abs(Mref @ x).max())


def test_pinv_preconditioner_symmetric_positive():
    mdl = small_model(ncomp=2, mask=True)
    M = precond.PseudoInversePrecond(mdl)
    n = mdl.n
    Mm = np.stack([M(e) for e in np.eye(n)], axis=1)
    assert np.max(np.abs(Mm - Mm.T)) < 1e-11 * np.abs(Mm).max()
    assert np.linalg.eigvalsh(0.5 * (Mm + Mm.T)).min() > 0


def test_diag_preconditioner_inverts_dense_diagonal_blocks():
    mdl = small_model(ncomp=2, mask=True)
    A = dense.dense_a(mdl)
    Md = precond.DiagonalPrecond(mdl)
    # brute force: for each (l, m, part) gather the N_comp x N_comp block of A
    lu = max(c["lmax"] for c in mdl.comps)
    ell_u, m_u, p_u = sht.lm_arrays(lu)
    rng = np.random.default_rng(9)
    r = rng.standard_normal(mdl.n)
    z = Md(r)
    zref = np.zeros(mdl.n)
    for i in range(len(ell_u)):
        l, m, p = ell_u[i], m_u[i], p_u[i]
        idx = [mdl.offsets[k] + sht.index(c["lmax"], l, m, p)
               for k, c in enumerate(mdl.comps) if l <= c["lmax"]]
        blk = A[np.ix_(idx, idx)]
        zref[idx] = np.linalg.solve(blk, r[idx])
    np.testing.assert_allclose(z, zref, rtol=1e-10, atol=1e-10 * np.abs(zref).max())


def test_pcg_matches_cholesky_tiny_workload():
    prob = inputs.make_problem("tiny")
    mdl, _ = oracle_model(prob)
    s, d = synthetic_data(prob, mdl)
    b = rhs.build_rhs(mdl, d=d)
    A = dense.dense_a(mdl)
    xref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), b)
    for M in (precond.PseudoInversePrecond(mdl), precond.DiagonalPrecond(mdl)):
        res = pcg.pcg(mdl.apply_A, M, b, rtol=1e-10, maxiter=500)
        assert res.status == "ok"
        assert np.linalg.norm(res.x - xref) / np.linalg.norm(xref) < 1e-8


def test_pcg_matches_cholesky_small_multires():
    prob = inputs.make_problem("multires", scale=16)  # Nside 4/8/8/16/16, L_k = 32
    mdl, _ = oracle_model(prob)
    assert [b["lmax"] for b in mdl.bands] == [8, 16, 16, 32, 32]
    rng = np.random.default_rng(3)
    xt = inputs.signal_coefficients(prob)
    b = mdl.apply_A(xt)
    A = dense.dense_a(mdl)
    xref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), b)
    assert np.linalg.norm(xref - xt) / np.linalg.norm(xt) < 1e-9
    Mp = precond.PseudoInversePrecond(mdl)
    Md = precond.DiagonalPrecond(mdl)
    rp = pcg.pcg(mdl.apply_A, Mp, b, rtol=1e-10, maxiter=500, x_true=xt)
    rd = pcg.pcg(mdl.apply_A, Md, b, rtol=1e-10, maxiter=500, x_true=xt)
    assert rp.status == "ok" and rd.status == "ok"
    assert np.linalg.norm(rp.x - xref) / np.linalg.norm(xref) < 1e-8
    # Sect. 3.3: with inhomogeneous noise on the full sky M_PI needs fewer iterations
    assert rp.iters <= rd.iters  # qualitative only at this tiny size


def test_pcg_reports_breakdown_on_indefinite_system():
    A = np.diag([1.0, -2.0, 3.0])
    res = pcg.pcg(lambda v: A @ v, lambda v: v, np.array([1.0, 1.0, 1.0]), rtol=1e-12)
    assert res.status == "breakdown"
    res = pcg.pcg(lambda v: v, lambda v: v * np.nan, np.ones(3))
    assert res.status == "breakdown"


def test_cr_rhs_covariance_equals_a():
    """Cov(b) = K K^T with K = [P^T N^-1/2, S^-1/2] must equal A (Sect. 2.3)."""
    mdl = small_model(ncomp=2, mask=True)
    A = dense.dense_a(mdl)
    cols = []
    for nu, b in enumerate(mdl.bands):
        for i in range(b["grid"].npix):
            e = np.zeros(b["grid"].npix)
            e[i] = 1.0
            om1 = [None] * len(mdl.bands)
            om1[nu] = e
            cols.append(rhs.build_rhs(mdl, omega1=om1))
    for i in range(mdl.n):
        e = np.zeros(mdl.n)
        e[i] = 1.0
        cols.append(rhs.build_rhs(mdl, omega2=e))
    K = np.stack(cols, axis=1)
    np.testing.assert_allclose(K @ K.T, A, atol=1e-11 * np.abs(A).max())


def _numpy_philox_block(counter, key):
    """numpy's Philox (4x64, 10 rounds) increments its 256-bit counter before
    each block, so start it one below the wanted counter."""
    c = sum(int(v) << (64 * i) for i, v in enumerate(counter)) - 1
    c %= 1 << 256
    start = [(c >> (64 * i)) & (2 ** 64 - 1) for i in range(4)]
    return np.random.Philox(counter=np.array(start, dtype=np.uint64),
                            key=np.array(key, dtype=np.uint64)).random_raw(4)


def test_philox_matches_numpy_bit_generator():
    for seed, stream, rhs_i in ((0, 0, 0), (12345, 0x203, 7), (2 ** 63 + 5, 1, 2 ** 40)):
        w = philox.raw_words(seed, stream, rhs_i, 12)
        for blk in range(3):
            ref = _numpy_philox_block([blk, rhs_i, 0, 0], [seed, stream])
            np.testing.assert_array_equal(w[4 * blk:4 * blk + 4], ref)


def test_normals_statistics():
    x = philox.normals(7, 0x100, 0, 200000)
    assert abs(x.mean()) < 0.01 and abs(x.var() - 1) < 0.01
    assert abs(np.mean(x ** 4) - 3) < 0.05


def test_uniform_words_closed_forms():
    """((w >> 11) + 0.5) 2^-53 at the ends of the 64-bit range and one step in."""
    u = philox.uniforms(np.array([0, 2 ** 64 - 1, 2 ** 11, 2 ** 63], dtype=np.uint64))
    assert u[0] == 2.0 ** -54
    assert u[1] == 1.0 - 2.0 ** -54
    assert u[2] == 1.5 * 2.0 ** -53
    assert u[3] == 0.5 + 2.0 ** -54


def test_box_muller_closed_forms():
    """Box and Muller (1958): X1 = sqrt(-2 ln U1) cos(2 pi U2), X2 = sqrt(-2 ln U1)
    sin(2 pi U2), evaluated at inputs whose outputs are known in closed form.
    Swapping cos and sin, or the roles of the two uniforms of a pair, or the
    pairing (u0, u1), (u2, u3), changes at least one of these values."""
    e2, eh = math.exp(-2.0), math.exp(-0.5)
    u = np.array([[e2, 1.0 / 12.0, eh, 0.25],
                  [e2, 0.5, eh, 0.125]])
    z = philox.box_muller(u)
    # radius sqrt(-2 ln e^-2) = 2 at angle pi/6; radius 1 at angle pi/2
    np.testing.assert_allclose(z[0], [math.sqrt(3.0), 1.0, 0.0, 1.0], atol=2e-15)
    # radius 2 at angle pi; radius 1 at angle pi/4
    np.testing.assert_allclose(z[1], [-2.0, 0.0, math.sqrt(0.5), math.sqrt(0.5)], atol=2e-15)
    # normals() is uniforms() then box_muller() on blocks of four words
    w = philox.raw_words(5, 0x101, 3, 8)
    ref = philox.box_muller(philox.uniforms(w).reshape(2, 4)).reshape(-1)
    np.testing.assert_array_equal(philox.normals(5, 0x101, 3, 8), ref)


def _twin_band_model(scale_tau=2.5, beam_other=None, seed=9):
    """Two components; band 1 is band 0 observed again (same grid, beam, SED)
    with its inverse noise scaled: rows of U proportional, normalised noise
    equal (the case of App. A.3)."""
    rng = np.random.default_rng(seed)
    g8, g4 = geometry.healpix(8), geometry.healpix(4)
    tau = np.exp(0.5 * rng.standard_normal(g8.npix))
    L = 12
    beam = inputs.gaussian_beam(400.0, L)
    bands = [{"grid": g8, "lmax": L, "beam": beam, "tau": tau},
             {"grid": g8, "lmax": L, "beam": beam if beam_other is None else beam_other,
              "tau": scale_tau * tau},
             {"grid": g4, "lmax": 8, "beam": inputs.gaussian_beam(600.0, 8),
              "tau": np.exp(0.5 * rng.standard_normal(g4.npix))}]
    comps = [{"lmax": 12, "invcl": inputs.inv_cl("cmb", 12, amplitude=0.05)},
             {"lmax": 12, "invcl": inputs.inv_cl("powerlaw", 12, amplitude=0.05)}]
    q = np.array([[1.0, 0.7], [1.0, 0.7], [1.0, 1.9]])
    return Model(bands, comps, q)


def test_merged_observations_leave_pinv_unchanged_for_twin_bands():
    """App. A.3: with U_2 = gamma U_1 and equal normalised noise the merged
    preconditioner (one row sqrt(1 + gamma^2) U_1, band 2's SHTs dropped) is
    the same operator as the unmerged one."""
    mdl = _twin_band_model()
    M0 = precond.PseudoInversePrecond(mdl)
    M1 = precond.PseudoInversePrecond(mdl, merge=[[0, 1]])
    assert M1.dropped == {1}
    r = np.random.default_rng(2).standard_normal((3, mdl.n))
    for v in r:
        np.testing.assert_allclose(M1(v), M0(v), rtol=1e-11, atol=1e-12 * np.abs(M0(v)).max())
    # gamma is the ratio of the rows: sqrt(alpha_2^2 / alpha_1^2) = sqrt(2.5)
    U = precond.u_blocks(mdl, M0.alpha2)
    Um = precond.merge_rows(U, 3, [[0, 1]])
    np.testing.assert_allclose(Um[5, 0], math.sqrt(1.0 + 2.5) * U[5, 0], rtol=1e-13)
    assert not np.any(Um[:, 1])


def test_merged_observations_are_a_preconditioner_for_near_twins():
    """Rows only nearly proportional (a slightly different beam): the merged
    operator is a compromise that stays symmetric positive definite and still
    solves the system."""
    L = 12
    mdl = _twin_band_model(beam_other=inputs.gaussian_beam(440.0, L))
    M1 = precond.PseudoInversePrecond(mdl, merge=[[0, 1]])
    n = mdl.n
    M = np.stack([M1(e) for e in np.eye(n)], axis=1)
    np.testing.assert_allclose(M, M.T, atol=1e-10 * np.abs(M).max())
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    b = mdl.apply_A(np.random.default_rng(5).standard_normal(n))
    res = pcg.pcg(mdl.apply_A, M1, b, rtol=1e-10, maxiter=500)
    assert res.status == "ok"


def _varmix_model(const=None, seed=13):
    """Two bands, two components; the synchrotron-like component's mixing in
    band 1 is a smooth map on a Gauss-Legendre grid (const: a flat map)."""
    rng = np.random.default_rng(seed)
    g8, g4 = geometry.healpix(8), geometry.healpix(4)
    L = 10
    bands = [{"grid": g8, "lmax": L, "beam": inputs.gaussian_beam(400.0, L),
              "tau": np.exp(0.4 * rng.standard_normal(g8.npix))},
             {"grid": g4, "lmax": 8, "beam": inputs.gaussian_beam(600.0, 8),
              "tau": np.exp(0.4 * rng.standard_normal(g4.npix))}]
    comps = [{"lmax": L, "invcl": inputs.inv_cl("cmb", L, amplitude=0.05)},
             {"lmax": L, "invcl": inputs.inv_cl("powerlaw", L, amplitude=0.05)}]
    q = np.array([[1.0, 0.8], [1.0, 1.7]])
    gq = geometry.gauss_legendre(L + 1, 2 * L + 1)
    z, phi = gq.pixel_centres()
    qmap = np.full(gq.npix, const) if const is not None else 1.7 * (1.0 + 0.3 * z + 0.2 * np.cos(phi) * (1 - z * z))
    return Model(bands, comps, q, mixing_maps={(1, 1): (gq, qmap)})


def test_flat_mixing_map_equals_scalar_mixing():
    """eq:Q with a flat map q on a Gauss-Legendre grid (exact quadrature at the
    band-limit, Y^T W Y = I) is the scalar mixing q I."""
    mdl = _varmix_model(const=1.7)
    ref = Model(mdl.bands, mdl.comps, mdl.q)
    x = np.random.default_rng(1).standard_normal(mdl.n)
    np.testing.assert_allclose(mdl.apply_A(x), ref.apply_A(x), rtol=1e-12, atol=1e-12 * np.abs(ref.apply_A(x)).max())


def test_varying_mixing_map_apply_a_matches_dense():
    """A with a spatially varying mixing map against the dense A built from the
    dense Y, Q~ = Y^T W Q Y, and its symmetry; the preconditioners use the
    scalar of eq:optimal-q."""
    mdl = _varmix_model()
    A = dense.dense_a(mdl)
    np.testing.assert_allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    x = np.random.default_rng(2).standard_normal(mdl.n)
    np.testing.assert_allclose(mdl.apply_A(x), A @ x, rtol=1e-11, atol=1e-12 * np.abs(A @ x).max())
    qmap = mdl.mixing_maps[(1, 1)][1]
    assert abs(precond.effective_q(mdl)[1, 1] - (qmap ** 2).sum() / qmap.sum()) < 1e-14
    b = A @ x
    res = pcg.pcg(mdl.apply_A, precond.PseudoInversePrecond(mdl), b, rtol=1e-11, maxiter=400)
    assert res.status == "ok"
    np.testing.assert_allclose(res.x, x, atol=1e-8 * np.abs(x).max())
