"""GPU parity of the system operators, preconditioners, PCG and the CR
right-hand side against the oracle (through the C ABI)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import dense, pcg, philox, precond, rhs, sht
from paper_1710_00621_amd import inputs
from tests.helpers import rel_max, oracle_model, synthetic_data

pytestmark = pytest.mark.gpu

OP_TOL = 1e-10    # operator applications (a few SHTs each)
SOL_TOL = 1e-8    # PCG solutions


def _setup():
    import torch
    from paper_1710_00621_amd import crsolve
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, crsolve


_rel = rel_max


_CACHE = {}


def _models(name, scale, diag=True):
    """(oracle model, GPU model, problem) built from the same tau maps."""
    key = (name, scale, diag)
    if key in _CACHE:
        return _CACHE[key]
    torch, crsolve = _setup()
    prob = inputs.make_problem(name, scale=scale)
    om, taus = oracle_model(prob)
    gm = crsolve.model_from_problem(prob, taus, diag=diag)
    _CACHE[key] = (om, gm, prob)
    return _CACHE[key]


SMALL = [("tiny", 1), ("multires", 16), ("masked", 32), ("diff", 32)]


@pytest.mark.parametrize("name,scale", SMALL)
def test_operators_match_oracle(name, scale):
    torch, crsolve = _setup()
    print(f"case operators {name} scale={scale}", flush=True)
    om, gm, prob = _models(name, scale)
    assert gm.n == om.n
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, om.n))
    xt = torch.tensor(x, device="cuda")
    got = gm.apply_A(xt).cpu().numpy()
    for i in range(2):
        assert _rel(got[i], om.apply_A(x[i])) < OP_TOL
    Mp = precond.PseudoInversePrecond(om)
    np.testing.assert_allclose(gm.alpha2(), Mp.alpha2, rtol=1e-12)
    got = gm.apply_pinv(xt).cpu().numpy()
    for i in range(2):
        assert _rel(got[i], Mp(x[i])) < OP_TOL
    Md = precond.DiagonalPrecond(om)
    got = gm.apply_diag(xt).cpu().numpy()
    for i in range(2):
        assert _rel(got[i], Md(x[i])) < OP_TOL


def test_tiny_pcg_matches_cholesky():
    """Tiny workload: both preconditioners to rel.res 1e-10 vs a dense Cholesky solve."""
    torch, crsolve = _setup()
    om, gm, prob = _models("tiny", 1)
    _, d = synthetic_data(prob, om)
    b = rhs.build_rhs(om, d=d)
    A = dense.dense_a(om)
    xref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), b)
    bt = torch.tensor(b, device="cuda")
    for pc in ("pinv", "diag"):
        x, info = gm.pcg(bt, precond=pc, rtol=1e-10, maxiter=500)
        assert info["relres"][0] <= 1e-10
        assert _rel(x.cpu().numpy(), xref) < SOL_TOL


def test_pcg_iterates_match_oracle():
    """Same algorithm on both sides: the k-th iterates agree element by element
    to 1e-8 for k <= 50 (the GPU solve stopped after k iterations), the residual
    histories agree, and the solutions agree to 1e-8 (both driven to 1e-12)."""
    torch, crsolve = _setup()
    om, gm, prob = _models("multires", 16)
    xt = inputs.signal_coefficients(prob)
    b = om.apply_A(xt)
    bt = torch.tensor(b, device="cuda")
    for pc, M in (("pinv", precond.PseudoInversePrecond(om)), ("diag", precond.DiagonalPrecond(om))):
        ref = pcg.pcg(om.apply_A, M, b, rtol=1e-12, maxiter=400, keep_iterates=50)
        x, info = gm.pcg(bt, precond=pc, rtol=1e-12, maxiter=400, history=True)
        assert ref.status == "ok"
        assert _rel(x.cpu().numpy(), ref.x) < SOL_TOL
        h = info["history"][:, 0]
        k = min(len(h), len(ref.history), 50)
        np.testing.assert_allclose(h[:k], ref.history[:k], rtol=1e-8)
        assert abs(info["iters"][0] - ref.iters) <= 2
        nk = len(ref.iterates)
        for k in sorted(set([1, 2, 3, 5, 8, 13, 21, 34, 50, nk]) & set(range(1, nk + 1))):
            xk, ik = gm.pcg(bt, precond=pc, rtol=1e-14, maxiter=k, raise_on_error=False)
            assert ik["iters"][0] == k
            err = _rel(xk.cpu().numpy(), ref.iterates[k - 1])
            assert err < SOL_TOL, (pc, k, err)
        print(f"{pc}: {nk} iterates compared, {ref.iters} iterations", flush=True)


def test_pcg_multiple_rhs_and_restart_from_x0():
    torch, crsolve = _setup()
    om, gm, prob = _models("diff", 32)
    rng = np.random.default_rng(4)
    xs = rng.standard_normal((3, om.n))
    bs = np.stack([om.apply_A(v) for v in xs])
    bt = torch.tensor(bs, device="cuda")
    x, info = gm.pcg(bt, precond="pinv", rtol=1e-10, maxiter=300)
    for i in range(3):
        assert _rel(x[i].cpu().numpy(), xs[i]) < SOL_TOL
    # warm start from the solution converges immediately
    x2, info2 = gm.pcg(bt, precond="pinv", rtol=1e-8, maxiter=300, x0=x)
    assert max(info2["iters"]) <= 1
    # b = 0 gives x = 0
    z, info3 = gm.pcg(torch.zeros_like(bt[:1]), precond="pinv", rtol=1e-8, maxiter=10)
    assert float(z.abs().max()) == 0.0


def test_philox_bit_exact_and_normals():
    torch, crsolve = _setup()
    for seed, stream, r in ((3, 0x100, 0), (2 ** 40 + 7, 0x200, 5)):
        got = crsolve.philox_normals(seed, stream, r, 1001).cpu().numpy()
        ref = philox.normals(seed, stream, r, 1001)
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-14)


def test_rhs_matches_oracle_masked():
    """CR right-hand side with explicit omegas on a masked model (tau = 0 in
    the mask), and the Wiener-filter right-hand side."""
    torch, crsolve = _setup()
    om, gm, prob = _models("masked", 32)
    _, d = synthetic_data(prob, om)
    om1, om2 = rhs.draw_omegas(om, 1234)
    bref = rhs.build_rhs(om, d=d, omega1=om1, omega2=om2)
    dt = [torch.tensor(v, device="cuda").unsqueeze(0) for v in d]
    w1 = [torch.tensor(v, device="cuda").unsqueeze(0) for v in om1]
    w2 = torch.tensor(om2, device="cuda").unsqueeze(0)
    b = gm.build_rhs(d=dt, omega1=w1, omega2=w2)[0].cpu().numpy()
    assert _rel(b, bref) < OP_TOL
    bwf = gm.build_rhs(d=dt)[0].cpu().numpy()
    assert _rel(bwf, rhs.build_rhs(om, d=d)) < OP_TOL


def test_constrained_realization_matches_oracle():
    """Omegas drawn on the device from the Philox streams; the oracle draws the
    same streams, builds b and solves."""
    torch, crsolve = _setup()
    om, gm, prob = _models("diff", 32)
    _, d = synthetic_data(prob, om)
    seed = 99
    om1, om2 = rhs.draw_omegas(om, seed)
    bref = rhs.build_rhs(om, d=d, omega1=om1, omega2=om2)
    ref = pcg.pcg(om.apply_A, precond.PseudoInversePrecond(om), bref, rtol=1e-12, maxiter=500)
    dt = [torch.tensor(v, device="cuda").unsqueeze(0) for v in d]
    x, info = gm.constrained_realization(dt, seed, mode="cr", precond="pinv", rtol=1e-12,
                                         maxiter=500)
    assert ref.status == "ok" and info["status"] == 0
    assert _rel(x[0].cpu().numpy(), ref.x) < SOL_TOL
    xw, infow = gm.constrained_realization(dt, seed, mode="wf", precond="diag", rtol=1e-12,
                                           maxiter=500)
    refw = pcg.pcg(om.apply_A, precond.DiagonalPrecond(om), rhs.build_rhs(om, d=d),
                   rtol=1e-12, maxiter=500)
    assert _rel(xw[0].cpu().numpy(), refw.x) < SOL_TOL


def test_masked_solve_residual():
    """Masked model: GPU solve to 1e-10, residual measured with the oracle's A."""
    torch, crsolve = _setup()
    om, gm, prob = _models("masked", 64)
    _, d = synthetic_data(prob, om)
    b = rhs.build_rhs(om, d=d)
    bt = torch.tensor(b, device="cuda")
    for pc in ("diag", "pinv"):
        x, info = gm.pcg(bt, precond=pc, rtol=1e-10, maxiter=5000)
        r = b - om.apply_A(x.cpu().numpy())
        assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10
        print(f"masked-64 {pc}: {info['iters'][0]} iterations", flush=True)


@pytest.mark.timeout(400)
def test_full_size_multires_apply_and_solve():
    """Full-size multi-resolution workload (Nside 64..256, L_k = 512): the GPU
    solution's residual measured with the oracle's A, and the GPU A against
    the oracle's A on that same vector (one oracle application, ~1 min)."""
    torch, crsolve = _setup()
    print("case full-size multires", flush=True)
    prob = inputs.make_problem("multires")
    om, taus = oracle_model(prob)
    gm = crsolve.model_from_problem(prob, taus, diag=True)
    xt = inputs.signal_coefficients(prob)
    bt = gm.apply_A(torch.tensor(xt, device="cuda"))
    xs, info = gm.pcg(bt, precond="pinv", rtol=1e-8, maxiter=500)
    print(f"multires full: pinv iters {info['iters'][0]}", flush=True)
    xg = xs.cpu().numpy()
    Ax_ref = om.apply_A(xg)
    Ax_gpu = gm.apply_A(xs).cpu().numpy()
    assert _rel(Ax_gpu, Ax_ref) < OP_TOL
    b = bt.cpu().numpy()
    assert np.linalg.norm(b - Ax_ref) / np.linalg.norm(b) <= 1.5e-8


@pytest.mark.timeout(900)
def test_full_size_masked_apply_sampled():
    """The masked constrained-realization workload at full size (9 bands at
    Nside 512 / 1024, L_k = 2000, 3 components, galactic cut plus 500 disks):
    A x on the GPU against the oracle's A x on sampled outputs.  x is nonzero
    at a few m only, so the oracle synthesises only those m; tau (lognormal
    noise, zero in the mask) couples every m, and the outputs at a few other
    m (including aliased ones from the short polar rings) are compared
    element by element."""
    torch, crsolve = _setup()
    print("case full-size masked apply_A, sampled m", flush=True)
    prob = inputs.make_problem("masked")
    om, taus = oracle_model(prob)
    print("oracle model ready", flush=True)
    gm = crsolve.model_from_problem(prob, taus, diag=False)
    print("GPU model ready", flush=True)
    ms_in = [0, 1, 7, 500, 1500, 1999, 2000]
    ms_out = [0, 3, 7, 999, 1500, 2000]
    rng = np.random.default_rng(11)
    x = np.zeros(om.n)
    keep = np.zeros(om.n, dtype=bool)
    for k, c in enumerate(om.comps):
        mm = sht.lm_arrays(c["lmax"])[1]
        sl = slice(om.offsets[k], om.offsets[k + 1])
        x[sl] = np.where(np.isin(mm, ms_in), rng.standard_normal(len(mm)), 0.0)
        keep[sl] = np.isin(mm, ms_out)
    y = gm.apply_A(torch.tensor(x, device="cuda")).cpu().numpy()
    print("GPU apply done", flush=True)
    yref = om.apply_A(x, ms_in=ms_in, ms_out=ms_out)
    err = _rel(y[keep], yref[keep])
    print(f"sampled outputs {int(keep.sum())}, max-abs rel error {err:.2e}", flush=True)
    assert err < OP_TOL


@pytest.mark.timeout(600)
def test_full_resolution_apply_sampled():
    """Full Planck-like resolution (Nside 1024 and 2048 bands, L_nu = 2048 and
    4096, three components at L_k = 6000): the lowest and highest band of the
    9-band recipe, A x on the GPU against the oracle's A x at a few m in and
    out, including m above the band-limits where only the prior acts."""
    torch, crsolve = _setup()
    print("case full-resolution apply_A, 2 bands, sampled m", flush=True)
    prob = inputs.make_problem("fullres")
    sub = dict(prob, bands=[prob["bands"][0], prob["bands"][8]], q=prob["q"][[0, 8]])
    om, taus = oracle_model(sub)
    gm = crsolve.model_from_problem(sub, taus, diag=False)
    mb, eb = gm.plan_bytes(1)
    print(f"models ready; planned tables {mb / 2**30:.2f} GiB, operator state {eb / 2**30:.2f} GiB", flush=True)
    ms_in = [0, 5, 2048, 4096, 6000]
    ms_out = [0, 3, 2048, 4095, 5999]
    rng = np.random.default_rng(12)
    x = np.zeros(om.n)
    keep = np.zeros(om.n, dtype=bool)
    for k, c in enumerate(om.comps):
        mm = sht.lm_arrays(c["lmax"])[1]
        sl = slice(om.offsets[k], om.offsets[k + 1])
        x[sl] = np.where(np.isin(mm, ms_in), rng.standard_normal(len(mm)), 0.0)
        keep[sl] = np.isin(mm, ms_out)
    y = gm.apply_A(torch.tensor(x, device="cuda")).cpu().numpy()
    print("GPU apply done", flush=True)
    yref = om.apply_A(x, ms_in=ms_in, ms_out=ms_out)
    err = _rel(y[keep], yref[keep])
    print(f"sampled outputs {int(keep.sum())}, max-abs rel error {err:.2e}", flush=True)
    assert err < OP_TOL


def _twin_models(beam_other_fwhm=None):
    """GPU and oracle copies of a model whose band 1 repeats band 0 (same grid,
    beam and SED, inverse noise scaled by 2.5); beam_other_fwhm gives band 1 a
    slightly different beam (a near twin)."""
    torch, crsolve = _setup()
    from oracle import geometry as ogeo
    from oracle.model import Model as OModel
    rng = np.random.default_rng(9)
    L = 12
    g8, g4 = crsolve.Grid.healpix(8), crsolve.Grid.healpix(4)
    o8, o4 = ogeo.healpix(8), ogeo.healpix(4)
    tau = np.exp(0.5 * rng.standard_normal(o8.npix))
    tau4 = np.exp(0.5 * rng.standard_normal(o4.npix))
    beam = inputs.gaussian_beam(400.0, L)
    beam1 = beam if beam_other_fwhm is None else inputs.gaussian_beam(beam_other_fwhm, L)
    beam4 = inputs.gaussian_beam(600.0, 8)
    comps = [{"lmax": 12, "invcl": inputs.inv_cl("cmb", 12, amplitude=0.05)},
             {"lmax": 12, "invcl": inputs.inv_cl("powerlaw", 12, amplitude=0.05)}]
    q = np.array([[1.0, 0.7], [1.0, 0.7], [1.0, 1.9]])
    spec = [(g8, o8, L, beam, tau), (g8, o8, L, beam1, 2.5 * tau), (g4, o4, 8, beam4, tau4)]
    gm = crsolve.Model([{"grid": g, "lmax": l, "beam": b, "tau": t} for g, _, l, b, t in spec], comps, q,
                       diag=True)
    om = OModel([{"grid": o, "lmax": l, "beam": b, "tau": t} for _, o, l, b, t in spec], comps, q)
    gm._keep_grids = (g8, g4)
    return om, gm


def test_merged_observations_match_oracle():
    """App. A.3 on the GPU: for twin bands the merged M_PI equals the unmerged
    one and runs fewer Legendre flops; for near twins it matches the oracle's
    merged operator, and a PCG solve with it matches the oracle's solve."""
    torch, crsolve = _setup()
    om, gm = _twin_models()
    x = np.random.default_rng(3).standard_normal((2, om.n))
    xt = torch.tensor(x, device="cuda")
    crsolve.kernel_stats_reset()
    crsolve.set_profiling(True)
    z0 = gm.apply_pinv(xt).cpu().numpy()
    torch.cuda.synchronize()
    w0 = crsolve.kernel_stats("legendre_synth")["work"]
    gm.merge_observations([[0, 1]])
    crsolve.kernel_stats_reset()
    z1 = gm.apply_pinv(xt).cpu().numpy()
    torch.cuda.synchronize()
    w1 = crsolve.kernel_stats("legendre_synth")["work"]
    crsolve.set_profiling(False)
    for i in range(2):
        assert _rel(z1[i], z0[i]) < 1e-11
    print(f"Legendre synthesis work unmerged {w0:.3e}, merged {w1:.3e}", flush=True)
    assert w1 < w0  # band 1's T^+ transforms are no longer run
    om2, gm2 = _twin_models(beam_other_fwhm=440.0)
    gm2.merge_observations([[0, 1]])
    Mref = precond.PseudoInversePrecond(om2, merge=[[0, 1]])
    z2 = gm2.apply_pinv(xt).cpu().numpy()
    for i in range(2):
        assert _rel(z2[i], Mref(x[i])) < OP_TOL
    b = om2.apply_A(x[0])
    ref = pcg.pcg(om2.apply_A, Mref, b, rtol=1e-12, maxiter=500)
    xs, info = gm2.pcg(torch.tensor(b, device="cuda"), precond="pinv", rtol=1e-12, maxiter=500)
    assert ref.status == "ok" and info["status"] == 0
    assert _rel(xs.cpu().numpy(), ref.x) < SOL_TOL
    assert abs(info["iters"][0] - ref.iters) <= 2


def _varmix_models(const=None, extra_pair=False):
    """GPU and oracle copies of a two-band, two-component model whose
    (band 1, component 1) mixing is a smooth map on a Gauss-Legendre grid
    (const: a flat map); extra_pair adds a HEALPix mixing map on (band 0, comp 1)."""
    torch, crsolve = _setup()
    from oracle import geometry as ogeo
    from oracle.model import Model as OModel
    rng = np.random.default_rng(13)
    L = 10
    o8, o4 = ogeo.healpix(8), ogeo.healpix(4)
    g8, g4 = crsolve.Grid.healpix(8), crsolve.Grid.healpix(4)
    t8 = np.exp(0.4 * rng.standard_normal(o8.npix))
    t4 = np.exp(0.4 * rng.standard_normal(o4.npix))
    comps = [{"lmax": L, "invcl": inputs.inv_cl("cmb", L, amplitude=0.05)},
             {"lmax": L, "invcl": inputs.inv_cl("powerlaw", L, amplitude=0.05)}]
    q = np.array([[1.0, 0.8], [1.0, 1.7]])
    spec = [(g8, o8, L, inputs.gaussian_beam(400.0, L), t8), (g4, o4, 8, inputs.gaussian_beam(600.0, 8), t4)]
    oq = ogeo.gauss_legendre(L + 1, 2 * L + 1)
    gq = crsolve.Grid.gauss_legendre(L + 1, 2 * L + 1)
    z, phi = oq.pixel_centres()
    qmap = np.full(oq.npix, const) if const is not None else \
        1.7 * (1.0 + 0.3 * z + 0.2 * np.cos(phi) * (1 - z * z))
    maps = {(1, 1): (oq, qmap)}
    gm = crsolve.Model([{"grid": g, "lmax": l, "beam": b, "tau": t} for g, _, l, b, t in spec], comps, q, diag=True)
    gm.set_mixing_map(1, 1, gq, qmap)
    if extra_pair:
        z8, phi8 = o8.pixel_centres()
        q8 = 0.8 * (1.0 - 0.25 * z8 * z8)
        maps[(0, 1)] = (o8, q8)
        gm.set_mixing_map(0, 1, g8, q8)
    om = OModel([{"grid": o, "lmax": l, "beam": b, "tau": t} for _, o, l, b, t in spec], comps, q, mixing_maps=maps)
    gm._keep_grids = (g8, g4, gq)
    return om, gm


@pytest.mark.parametrize("extra", [False, True])
def test_varying_mixing_maps_match_oracle(extra):
    """eq:Q on the GPU: A, the right-hand side, P x and both preconditioners
    (with the eq:optimal-q scalar) against the oracle element by element, and
    a PCG solve to 1e-12; a flat map equals scalar mixing."""
    torch, crsolve = _setup()
    om, gm = _varmix_models(extra_pair=extra)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, om.n))
    xt = torch.tensor(x, device="cuda")
    y = gm.apply_A(xt).cpu().numpy()
    zp = gm.apply_pinv(xt).cpu().numpy()
    zd = gm.apply_diag(xt).cpu().numpy()
    Mp, Md = precond.PseudoInversePrecond(om), precond.DiagonalPrecond(om)
    for i in range(2):
        assert _rel(y[i], om.apply_A(x[i])) < OP_TOL
        assert _rel(zp[i], Mp(x[i])) < OP_TOL
        assert _rel(zd[i], Md(x[i])) < OP_TOL
    maps = gm.project(xt[0])
    for nu in range(2):
        assert _rel(maps[nu].cpu().numpy(), om.project(x[0], nu)) < OP_TOL
    d = [rng.standard_normal(b["grid"].npix) for b in om.bands]
    b = gm.build_rhs(d=[torch.tensor(v, device="cuda").unsqueeze(0) for v in d])[0].cpu().numpy()
    bref = rhs.build_rhs(om, d=d)
    assert _rel(b, bref) < OP_TOL
    ref = pcg.pcg(om.apply_A, Mp, bref, rtol=1e-12, maxiter=500)
    xs, info = gm.pcg(torch.tensor(bref, device="cuda"), precond="pinv", rtol=1e-12, maxiter=500)
    assert ref.status == "ok" and info["status"] == 0
    assert _rel(xs.cpu().numpy(), ref.x) < SOL_TOL
    assert abs(info["iters"][0] - ref.iters) <= 2
    if not extra:
        om_c, gm_c = _varmix_models(const=1.7)
        scal = crsolve.Model([{"grid": g, "lmax": l, "beam": bb, "tau": t}
                              for g, (l, bb, t) in zip(gm_c._keep_grids[:2],
                                                       [(b_["lmax"], b_["beam"], b_["tau"]) for b_ in om_c.bands])],
                             om_c.comps, om_c.q, diag=False)
        assert _rel(gm_c.apply_A(xt).cpu().numpy(), scal.apply_A(xt).cpu().numpy()) < 1e-12
