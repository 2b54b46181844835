"""GPU mask-restricted preconditioner (M_mask, multigrid V-cycle of Sect. 4.4)
and M_add = M_PI + M_mask against the oracle (through the C ABI)."""
import numpy as np
import pytest

from oracle import mask, pcg, precond, rhs
from paper_1710_00621_amd import inputs
from tests.helpers import oracle_model, rel_max, synthetic_data

pytestmark = pytest.mark.gpu

CASES = [("masked", 16, 0), ("batched", 2, 0), ("batched", 4, 5), ("batched", 2, 7)]
# small enough for the oracle's M_add solve to take well under a minute or two
PCG_CASES = [("batched", 4, 3), ("batched", 8, 2)]
_CACHE = {}


def _setup():
    import torch
    from paper_1710_00621_amd import crsolve
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, crsolve


def _case(name, scale, index):
    key = (name, scale, index)
    if key in _CACHE:
        return _CACHE[key]
    torch, crsolve = _setup()
    prob = inputs.make_problem(name, scale=scale, index=index)
    om, taus = oracle_model(prob)
    grids = {}
    gl = []
    for b in prob["bands"]:
        if b["grid"] not in grids:
            grids[b["grid"]] = crsolve.Grid.from_spec(b["grid"])
        gl.append(grids[b["grid"]])
    gm = crsolve.model_from_problem(prob, taus, gl, diag=True)
    mgrid, m = crsolve.mask_of_problem(prob, taus, gl)
    gm.set_mask(mgrid, m)
    nside = mgrid.spec[1]
    Mm = mask.MaskPrecond(om, nside, m)
    _CACHE[key] = (prob, om, gm, Mm, taus, grids)
    return _CACHE[key]


@pytest.mark.parametrize("name,scale,index", CASES)
def test_mask_hierarchy_matches_oracle(name, scale, index):
    prob, om, gm, Mm, _, _ = _case(name, scale, index)
    ref = [(l.nside, l.lmax, len(l.idx)) for l in Mm.comp[0][0]]
    got = gm.mask_info()
    print(f"{name}/{scale}/{index}: levels {got}", flush=True)
    assert got == ref


@pytest.mark.parametrize("name,scale,index", CASES)
def test_apply_mask_matches_oracle(name, scale, index):
    """z = M_mask r for two right-hand sides, element by element."""
    torch, crsolve = _setup()
    print(f"case apply_mask {name} scale {scale} index {index}", flush=True)
    prob, om, gm, Mm, _, _ = _case(name, scale, index)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, om.n))
    got = gm.apply_mask(torch.tensor(x, device="cuda")).cpu().numpy()
    for i in range(2):
        ref = Mm(x[i])
        err = rel_max(got[i], ref)
        print(f"  rhs {i}: max-abs rel error {err:.2e}", flush=True)
        assert err < 1e-9


@pytest.mark.parametrize("name,scale,index", PCG_CASES)
def test_pcg_add_matches_oracle(name, scale, index):
    """Constrained realization with M_add to rel.res 1e-12 on both sides: the
    solutions agree to 1e-8 element by element and the iteration counts are
    the same algorithm's (within 2)."""
    torch, crsolve = _setup()
    print(f"case pcg M_add {name} scale {scale} index {index}", flush=True)
    prob, om, gm, Mm, taus, _ = _case(name, scale, index)
    _, d = synthetic_data(prob, om)
    seed = 4242
    w1, w2 = rhs.draw_omegas(om, seed)
    b = rhs.build_rhs(om, d=d, omega1=w1, omega2=w2)
    ref = pcg.pcg(om.apply_A, mask.AddPrecond(precond.PseudoInversePrecond(om), Mm), b, rtol=1e-12,
                  maxiter=2000)
    assert ref.status == "ok"
    dt = [torch.tensor(v, device="cuda").unsqueeze(0) for v in d]
    x, info = gm.constrained_realization(dt, seed, mode="cr", precond="add", rtol=1e-12, maxiter=2000)
    err = rel_max(x[0].cpu().numpy(), ref.x)
    print(f"  iterations gpu {info['iters'][0]} oracle {ref.iters}; max-abs rel {err:.2e}", flush=True)
    assert err < 1e-8
    assert abs(info["iters"][0] - ref.iters) <= 2


@pytest.mark.parametrize("name,scale,index", [("batched", 4, 5), ("masked", 16, 0)])
def test_apply_mask_exact_j_matches_oracle(name, scale, index):
    """The cycle with J = Y^T W Y applied exactly (crs_mask_opts.exact_j)
    against the oracle's cycle with exact J, element by element, and that
    cycle's symmetry <M a, b> = <a, M b>."""
    torch, crsolve = _setup()
    print(f"case apply_mask exact J {name} scale {scale} index {index}", flush=True)
    prob, om, _, _, taus, grids = _case(name, scale, index)
    gl = [grids[b["grid"]] for b in prob["bands"]]
    gm = crsolve.model_from_problem(prob, taus, gl, diag=False)
    mgrid, m = crsolve.mask_of_problem(prob, taus, gl)
    gm.set_mask(mgrid, m, exact_j=True)
    Mj = mask.MaskPrecond(om, mgrid.spec[1], m, exact_j=True)
    rng = np.random.default_rng(8)
    x = rng.standard_normal((2, om.n))
    got = gm.apply_mask(torch.tensor(x, device="cuda")).cpu().numpy()
    for i in range(2):
        ref = Mj(x[i])
        err = rel_max(got[i], ref)
        print(f"  rhs {i}: max-abs rel error {err:.2e}", flush=True)
        assert err < 1e-9
    sym = abs(got[0] @ x[1] - x[0] @ got[1]) / (abs(got[0] @ x[1]) + 1e-300)
    print(f"  symmetry defect {sym:.2e}", flush=True)
    assert sym < 1e-10


def test_batch_add_matches_per_model_solves():
    """M_add through a batch of small problems (graphs and no graphs) equals
    each model's own M_add solve."""
    torch, crsolve = _setup()
    print("case batch M_add", flush=True)
    grids, models, data, probs = {}, [], [], []
    for i in range(4):
        prob = inputs.make_problem("batched", scale=8, index=i)
        om, taus = oracle_model(prob)
        gl = []
        for b in prob["bands"]:
            if b["grid"] not in grids:
                grids[b["grid"]] = crsolve.Grid.from_spec(b["grid"])
            gl.append(grids[b["grid"]])
        m = crsolve.model_from_problem(prob, taus, gl, diag=False)
        mg, mk = crsolve.mask_of_problem(prob, taus, gl)
        m.set_mask(mg, mk)
        _, d = synthetic_data(prob, om)
        models.append(m)
        probs.append(prob)
        data.append([torch.tensor(v, device="cuda") for v in d])
    seeds = [77 + i for i in range(4)]
    batch = crsolve.Batch(models)
    xg, ig = batch.solve(d=data, seeds=seeds, mode="cr", precond="add", rtol=1e-11, maxiter=3000, use_graph=True)
    xp, ip = batch.solve(d=data, seeds=seeds, mode="cr", precond="add", rtol=1e-11, maxiter=3000, use_graph=False)
    assert ig["status"] == 0 and ip["status"] == 0
    for p, m in enumerate(models):
        xr, ir = m.constrained_realization([t.unsqueeze(0) for t in data[p]], seeds[p], mode="cr",
                                           precond="add", rtol=1e-11, maxiter=3000)
        a, b, c = xg[p].cpu().numpy(), xp[p].cpu().numpy(), xr[0].cpu().numpy()
        print(f"problem {p}: iterations batch {ig['iters'][p]} model {ir['iters'][0]}", flush=True)
        assert rel_max(a, c) < 1e-8 and rel_max(b, c) < 1e-8
        assert abs(ig["iters"][p] - ir["iters"][0]) <= 1
