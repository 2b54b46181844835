"""GPU differentiation: autograd Functions over the transforms and the solve,
checked against the oracle's implicit gradients and against central finite
differences of GPU solves."""
import math

import numpy as np
import pytest

from oracle import geometry, gradient, pcg, precond, sht
from paper_1710_00621_amd import inputs
from tests.helpers import rel_max, oracle_model

pytestmark = pytest.mark.gpu


def _setup():
    import torch
    from paper_1710_00621_amd import autograd, crsolve
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, crsolve, autograd


_rel = rel_max


def _data(prob, om, seed=17):
    rng = np.random.default_rng(seed)
    s = inputs.signal_coefficients(prob)
    return [om.project(s, nu) + rng.standard_normal(b["grid"].npix) / np.sqrt(b["tau"])
            for nu, b in enumerate(om.bands)]


def test_sht_backward_is_the_adjoint():
    torch, crsolve, autograd = _setup()
    g = crsolve.Grid.healpix(16)
    og = geometry.healpix(16)
    L = 24
    rng = np.random.default_rng(3)
    a = torch.tensor(rng.standard_normal(sht.nalm(L)), device="cuda", requires_grad=True)
    w = rng.standard_normal(og.npix)
    y = autograd.sht_synth(a, g, L)
    (y * torch.tensor(w, device="cuda")).sum().backward()
    assert _rel(a.grad.cpu().numpy(), sht.adjoint(og, L, w)) < 1e-10
    f = torch.tensor(rng.standard_normal(og.npix), device="cuda", requires_grad=True)
    v = rng.standard_normal(sht.nalm(L))
    (autograd.sht_adjoint(f, g, L) * torch.tensor(v, device="cuda")).sum().backward()
    assert _rel(f.grad.cpu().numpy(), sht.synth(og, L, v)) < 1e-10


def _diff_models(scale):
    torch, crsolve, autograd = _setup()
    prob = inputs.make_problem("diff", scale=scale)
    om, taus = oracle_model(prob)
    gm = crsolve.model_from_problem(prob, taus, diag=False)
    return prob, om, gm


def test_mixing_gradient_blocks_match_oracle():
    """apply_dA_dmix, apply_db_dmix and apply_prior_inv against the oracle's
    band-space formulas on the 7-band, 3-component model at Nside 16."""
    torch, crsolve, autograd = _setup()
    prob, om, gm = _diff_models(16)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(om.n)
    lam = rng.standard_normal(om.n)
    d = [rng.standard_normal(b["grid"].npix) for b in om.bands]
    xt, lt = torch.tensor(x, device="cuda"), torch.tensor(lam, device="cuda")
    dA = autograd.dA_dmix(gm, lt, xt).cpu().numpy()
    db = autograd.db_dmix(gm, lt, [torch.tensor(v, device="cuda") for v in d]).cpu().numpy()
    xs, ls = om.split(x), om.split(lam)
    refA = np.zeros_like(dA)
    refb = np.zeros_like(db)
    for nu, b in enumerate(om.bands):
        vx = gradient.band_adjoint(om, nu, b["tau"] * om.project(x, nu))
        vl = gradient.band_adjoint(om, nu, b["tau"] * om.project(lam, nu))
        vd = gradient.band_adjoint(om, nu, b["tau"] * d[nu])
        for k in range(len(om.comps)):
            refA[nu, k] = -(gradient.band_dot(om, nu, vx, k, ls[k]) + gradient.band_dot(om, nu, vl, k, xs[k]))
            refb[nu, k] = gradient.band_dot(om, nu, vd, k, ls[k])
    assert _rel(dA, refA) < 1e-10
    assert _rel(db, refb) < 1e-10
    assert _rel(autograd.prior_inv(gm, xt).cpu().numpy(), om.apply_prior_inv(x)) < 1e-13


def _beta_of(prob):
    return [c.get("beta", 0.0) for c in prob["comps"]]


def _gpu_loss(torch, autograd, prob, gm, d, beta, rtol):
    freqs = [b["freq"] for b in prob["bands"]]
    bt = torch.tensor(beta, dtype=torch.float64, device="cuda", requires_grad=True)
    dt = [torch.tensor(v, device="cuda", requires_grad=True) for v in d]
    q = autograd.mixing_matrix(freqs, prob["comps"], bt)
    loss, x = autograd.wf_loss(gm, dt, q, {"precond": "pinv", "rtol": rtol, "maxiter": 5000})
    return loss, bt, dt, x


def test_wf_loss_gradient_matches_oracle():
    """Loss, dL/dbeta and dL/dd of the Wiener-filter loss (7 bands at Nside
    16, CMB + synchrotron + dust) against the oracle's implicit gradient."""
    torch, crsolve, autograd = _setup()
    prob, om, gm = _diff_models(16)
    d = _data(prob, om)
    beta = _beta_of(prob)
    loss, bt, dt, x = _gpu_loss(torch, autograd, prob, gm, d, beta, 1e-12)
    loss.backward()
    Mp = precond.PseudoInversePrecond(om)

    def solve(v):
        r = pcg.pcg(om.apply_A, Mp, v, rtol=1e-12, maxiter=2000)
        assert r.status == "ok"
        return r.x

    L0, gd, gq, xo = gradient.wf_loss_and_gradient(om, d, solve)
    assert abs(float(loss) - L0) <= 1e-10 * abs(L0)
    assert _rel(x.detach().cpu().numpy(), xo) < 1e-8
    freqs = [b["freq"] for b in prob["bands"]]
    for k, c in enumerate(prob["comps"]):
        if c["kind"] == "cmb":
            continue
        ref = sum(gq[nu, k] * gradient.sed_dbeta(c["kind"], f, beta[k], c["nu_ref"], c.get("T", 20.0))
                  for nu, f in enumerate(freqs))
        assert abs(float(bt.grad[k]) - ref) <= 1e-7 * abs(ref), (k, float(bt.grad[k]), ref)
    for nu in range(len(d)):
        assert _rel(dt[nu].grad.cpu().numpy(), gd[nu]) < 1e-7


@pytest.mark.timeout(300)
def test_beta_gradient_matches_finite_differences():
    """Central differences (h = 1e-6 on beta, solves to rel.res 1e-13) of the
    GPU loss against its autograd gradient, 7 bands at Nside 32, L = 64."""
    torch, crsolve, autograd = _setup()
    print("case FD beta, diff scale 8", flush=True)
    prob, om, gm = _diff_models(8)
    d = _data(prob, om)
    beta = _beta_of(prob)
    loss, bt, dt, x = _gpu_loss(torch, autograd, prob, gm, d, beta, 1e-13)
    loss.backward()
    for k, c in enumerate(prob["comps"]):
        if c["kind"] == "cmb":
            continue
        h = 1e-6
        vals = []
        for sgn in (1.0, -1.0):
            b2 = list(beta)
            b2[k] += sgn * h
            with torch.no_grad():
                lv, _, _, _ = _gpu_loss(torch, autograd, prob, gm, d, b2, 1e-13)
            vals.append(float(lv))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(float(bt.grad[k]) - fd) <= 1e-5 * abs(fd), (k, float(bt.grad[k]), fd)
        print(f"beta[{k}]: autograd {float(bt.grad[k]):.10e} FD {fd:.10e}", flush=True)


def test_loss_terms_match_oracle():
    """The loss terms behind the C ABI (prior quadratic, chi-square with its
    residual maps, noise weighting) against the oracle at Nside 16."""
    torch, crsolve, autograd = _setup()
    prob, om, gm = _diff_models(16)
    rng = np.random.default_rng(8)
    x = rng.standard_normal((2, om.n))
    d = [rng.standard_normal((2, b["grid"].npix)) for b in om.bands]
    xt = torch.tensor(x, device="cuda")
    val, y = gm.prior_quad(xt)
    for r in range(2):
        Sx = om.apply_prior_inv(x[r])
        assert _rel(y[r].cpu().numpy(), Sx) < 1e-14
        assert abs(float(val[r]) - 0.5 * x[r] @ Sx) <= 1e-12 * abs(0.5 * x[r] @ Sx)
    chi, res = gm.chi2(xt, [torch.tensor(v, device="cuda") for v in d])
    for r in range(2):
        ref_res = [d[nu][r] - om.project(x[r], nu) for nu in range(len(om.bands))]
        ref = sum(float(rr @ (b["tau"] * rr)) for rr, b in zip(ref_res, om.bands))
        assert abs(float(chi[r]) - ref) <= 1e-11 * abs(ref)
        for nu in range(len(om.bands)):
            assert _rel(res[nu][r].cpu().numpy(), ref_res[nu]) < 1e-10
    w = gm.noise_weight([torch.tensor(v, device="cuda") for v in d], scale=2.0)
    for nu, b in enumerate(om.bands):
        assert _rel(w[nu].cpu().numpy(), 2.0 * b["tau"][None, :] * d[nu]) < 1e-15


def test_two_forwards_one_backward():
    """Two losses at different beta on the same model, summed, one backward:
    each beta's gradient matches central differences at its own beta (the
    backward passes restore the mixing matrix their forward used)."""
    torch, crsolve, autograd = _setup()
    prob, om, gm = _diff_models(16)
    d = _data(prob, om)
    b1 = _beta_of(prob)
    b2 = [b + (0.3 if i else 0.0) for i, b in enumerate(b1)]
    l1, bt1, _, _ = _gpu_loss(torch, autograd, prob, gm, d, b1, 1e-13)
    l2, bt2, _, _ = _gpu_loss(torch, autograd, prob, gm, d, b2, 1e-13)
    (l1 + l2).backward()
    for beta, bt in ((b1, bt1), (b2, bt2)):
        for k, c in enumerate(prob["comps"]):
            if c["kind"] == "cmb":
                continue
            h = 1e-6
            vals = []
            for sgn in (1.0, -1.0):
                bb = list(beta)
                bb[k] += sgn * h
                with torch.no_grad():
                    lv, _, _, _ = _gpu_loss(torch, autograd, prob, gm, d, bb, 1e-13)
                vals.append(float(lv))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(float(bt.grad[k]) - fd) <= 1e-5 * abs(fd), (beta, k, float(bt.grad[k]), fd)


@pytest.mark.timeout(600)
def test_full_size_gradients_match_finite_differences():
    """The differentiation workload at full size (7 bands at Nside 256, L = 512,
    CMB + synchrotron + dust): dL/dbeta by the implicit backward against
    central differences (h = 1e-6, solves to rel.res 1e-13), and dL/dd along
    two random unit directions in data space.  The loss is quadratic in d (x is
    linear in d), so a central difference along d is exact for any step: h = 1
    there keeps the difference far above the rounding of a loss of ~5e6."""
    torch, crsolve, autograd = _setup()
    print("case full-size gradients", flush=True)
    prob = inputs.make_problem("diff")
    taus = inputs.inverse_noise_maps(prob, None)
    gm = crsolve.model_from_problem(prob, taus, diag=False)
    rng = np.random.default_rng(19)
    s = torch.tensor(inputs.signal_coefficients(prob), device="cuda")
    sig = gm.project(s)
    d = [(sig[nu][0] + torch.tensor(rng.standard_normal(len(t)) / np.sqrt(t), device="cuda")).cpu().numpy()
         for nu, t in enumerate(taus)]
    beta = _beta_of(prob)
    loss, bt, dt, x = _gpu_loss(torch, autograd, prob, gm, d, beta, 1e-13)
    loss.backward()
    print(f"loss {float(loss):.6e}", flush=True)
    h = 1e-6
    for k, c in enumerate(prob["comps"]):
        if c["kind"] == "cmb":
            continue
        vals = []
        for sgn in (1.0, -1.0):
            b2 = list(beta)
            b2[k] += sgn * h
            with torch.no_grad():
                lv, _, _, _ = _gpu_loss(torch, autograd, prob, gm, d, b2, 1e-13)
            vals.append(float(lv))
        fd = (vals[0] - vals[1]) / (2 * h)
        print(f"beta[{k}]: autograd {float(bt.grad[k]):.10e} FD {fd:.10e}", flush=True)
        assert abs(float(bt.grad[k]) - fd) <= 1e-5 * abs(fd), (k, float(bt.grad[k]), fd)
    for j in range(2):
        u = [rng.standard_normal(len(v)) for v in d]
        nrm = math.sqrt(sum(float(v @ v) for v in u))
        u = [v / nrm for v in u]
        g_dir = sum(float(dt[nu].grad.cpu().numpy() @ u[nu]) for nu in range(len(d)))
        vals = []
        hd = 1.0
        for sgn in (1.0, -1.0):
            d2 = [v + sgn * hd * w for v, w in zip(d, u)]
            with torch.no_grad():
                lv, _, _, _ = _gpu_loss(torch, autograd, prob, gm, d2, beta, 1e-13)
            vals.append(float(lv))
        fd = (vals[0] - vals[1]) / (2 * hd)
        print(f"d direction {j}: autograd {g_dir:.10e} FD {fd:.10e}", flush=True)
        assert abs(g_dir - fd) <= 1e-5 * abs(fd), (j, g_dir, fd)
