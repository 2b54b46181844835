"""GPU batch of many problems (stacked PCG, shared transform launches, one
hipGraph per iteration) against the per-model solves and the oracle."""
import numpy as np
import pytest

from oracle import pcg, precond, rhs
from paper_1710_00621_amd import inputs
from tests.helpers import oracle_model, synthetic_data

pytestmark = pytest.mark.gpu

SOL_TOL = 1e-8


def _setup():
    import torch
    from paper_1710_00621_amd import crsolve
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, crsolve


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


_CACHE = {}


def _batch_setup(nprob, scale):
    key = (nprob, scale)
    if key in _CACHE:
        return _CACHE[key]
    torch, crsolve = _setup()
    grids = {}
    probs, oms, models, data = [], [], [], []
    for i in range(nprob):
        prob = inputs.make_problem("batched", scale=scale, index=i)
        om, taus = oracle_model(prob)
        gl = []
        for b in prob["bands"]:
            if b["grid"] not in grids:
                grids[b["grid"]] = crsolve.Grid.from_spec(b["grid"])
            gl.append(grids[b["grid"]])
        models.append(crsolve.model_from_problem(prob, taus, grids=gl, diag=False))
        _, d = synthetic_data(prob, om)
        probs.append(prob)
        oms.append(om)
        data.append([torch.tensor(v, device="cuda") for v in d])
    _CACHE[key] = (probs, oms, models, data, grids)
    return _CACHE[key]


def test_batch_matches_per_model_solves():
    """Six problems of three shapes (1-2 components, masks): the batched CR
    solve, with and without graphs, equals each model's own solve."""
    torch, crsolve = _setup()
    print("case batch vs per-model, 6 problems, scale 8", flush=True)
    probs, oms, models, data, _ = _batch_setup(6, 8)
    seeds = [1000 + i for i in range(len(models))]
    batch = crsolve.Batch(models)
    xg, infog = batch.solve(d=data, seeds=seeds, mode="cr", precond="pinv", rtol=1e-10,
                            maxiter=3000, use_graph=True)
    xp, infop = batch.solve(d=data, seeds=seeds, mode="cr", precond="pinv", rtol=1e-10,
                            maxiter=3000, use_graph=False)
    assert infog["status"] == 0 and infop["status"] == 0
    for p, m in enumerate(models):
        xr, info = m.constrained_realization([t.unsqueeze(0) for t in data[p]], seeds[p], mode="cr",
                                             precond="pinv", rtol=1e-10, maxiter=3000)
        assert info["status"] == 0
        a, b, c = xg[p].cpu().numpy(), xp[p].cpu().numpy(), xr[0].cpu().numpy()
        assert _rel(a, c) < SOL_TOL, p
        assert _rel(b, c) < SOL_TOL, p
        assert infog["relres"][p] <= 1e-10
        # same arithmetic per problem: the iteration counts agree
        assert abs(infog["iters"][p] - info["iters"][0]) <= 1, (p, infog["iters"][p], info["iters"][0])
        print(f"problem {p}: {infog['iters'][p]} iterations", flush=True)


def test_batch_problem_matches_oracle():
    """One problem of the batch against the oracle's CR solve with the same
    Philox draws (both driven to 1e-12)."""
    torch, crsolve = _setup()
    probs, oms, models, data, _ = _batch_setup(6, 8)
    seeds = [2000 + i for i in range(len(models))]
    batch = crsolve.Batch(models)
    xs, info = batch.solve(d=data, seeds=seeds, mode="cr", precond="pinv", rtol=1e-12,
                           maxiter=5000, use_graph=True)
    for p in (0, 3):
        om = oms[p]
        w1, w2 = rhs.draw_omegas(om, seeds[p])
        b = rhs.build_rhs(om, d=[t.cpu().numpy() for t in data[p]], omega1=w1, omega2=w2)
        ref = pcg.pcg(om.apply_A, precond.PseudoInversePrecond(om), b, rtol=1e-12, maxiter=5000)
        assert ref.status == "ok"
        assert _rel(xs[p].cpu().numpy(), ref.x) < SOL_TOL, p


def test_batch_wf_and_profiling_in_graphs():
    """Wiener filter through the batch (graph path) with profiling on: the
    kernel statistics see the launches inside the graphs, and the result
    matches the per-model Wiener filter."""
    torch, crsolve = _setup()
    probs, oms, models, data, _ = _batch_setup(6, 8)
    batch = crsolve.Batch(models)
    crsolve.kernel_stats_reset()
    crsolve.set_profiling(True)
    try:
        xs, info = batch.solve(d=data, mode="wf", precond="pinv", rtol=1e-10, maxiter=3000,
                               use_graph=True)
        st = crsolve.kernel_stats("legendre_synth")
    finally:
        crsolve.set_profiling(False)
    assert info["status"] == 0
    assert st["launches"] > 0 and st["ms"] > 0
    for p in (1, 5):
        xr, _ = models[p].constrained_realization([t.unsqueeze(0) for t in data[p]], 0, mode="wf",
                                                  precond="pinv", rtol=1e-10, maxiter=3000)
        assert _rel(xs[p].cpu().numpy(), xr[0].cpu().numpy()) < SOL_TOL
