"""GPU batch of many problems (stacked PCG, shared transform launches, one
hipGraph per iteration) against the per-model solves and the oracle."""
import numpy as np
import pytest

from oracle import pcg, precond, rhs
from paper_1710_00621_amd import inputs
from tests.helpers import rel_max, oracle_model, synthetic_data

pytestmark = pytest.mark.gpu

SOL_TOL = 1e-8


def _setup():
    import torch
    from paper_1710_00621_amd import crsolve
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, crsolve


_rel = rel_max


_CACHE = {}


def _batch_setup(nprob, scale, diag=False):
    key = (nprob, scale, diag)
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
        models.append(crsolve.model_from_problem(prob, taus, grids=gl, diag=diag))
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


def test_batch_group_streams_bitwise():
    """Transform groups on four streams (graphs and the plain loop) give the
    bitwise result of one stream: each group writes its own buffers and the
    back-mix sums them in a fixed order after the join."""
    torch, crsolve = _setup()
    print("case batch group streams 1 vs 4, 6 problems, scale 8", flush=True)
    probs, oms, models, data, _ = _batch_setup(6, 8, diag=True)
    seeds = [1100 + i for i in range(len(models))]
    batch = crsolve.Batch(models)
    out = {}
    for ns in (1, 4):
        batch.set_streams(ns)
        for g in (True, False):
            x, info = batch.solve(d=data, seeds=seeds, mode="cr", precond="diag", rtol=1e-9,
                                  maxiter=3000, use_graph=g)
            assert info["status"] == 0
            out[(ns, g)] = ([t.cpu().numpy() for t in x], list(info["iters"]))
    for g in (True, False):
        (x1, i1), (x4, i4) = out[(1, g)], out[(4, g)]
        assert i1 == i4
        for a, b in zip(x1, x4):
            np.testing.assert_array_equal(a, b)
    with pytest.raises(Exception):
        batch.set_streams(9)


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


def _with_env(env, fn):
    import os
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return fn()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("forced", [None, "mfma2"])
def test_batch_diag_matches_oracle(forced):
    """Block-diagonal preconditioner through the batch (the benchmark's
    configuration) at 1/8 scale: six CR problems of three shapes (masks, 1-3
    components), with and without graphs, each against the oracle's M_diag
    PCG on the same Philox draws (both driven to 1e-12).  "mfma2" forces the
    matrix-core Legendre kernels with two 64-pair tiles per adjoint wave in
    every group (the variant the autotuner picks for the large groups)."""
    torch, crsolve = _setup()
    print(f"case batch diag vs oracle, forced={forced}", flush=True)
    probs, oms, models, data, _ = _batch_setup(6, 8, diag=True)
    seeds = [3000 + i for i in range(len(models))]
    env = {"CRS_LEG_MFMA_MIN": "1", "CRS_LEG_TA": "2"} if forced else {}
    batch = _with_env(env, lambda: crsolve.Batch(models))
    xg, infog = batch.solve(d=data, seeds=seeds, mode="cr", precond="diag", rtol=1e-12,
                            maxiter=5000, use_graph=True)
    st = batch.stats()
    # chunks of 8 iterations per graph launch, the host reading flags between them
    assert st["iterations"] == max(infog["iters"])
    assert st["graph_launches"] <= (st["iterations"] + 7) // 8 + 8, st
    print(f"graph stats {st}", flush=True)
    xp, infop = batch.solve(d=data, seeds=seeds, mode="cr", precond="diag", rtol=1e-12,
                            maxiter=5000, use_graph=False)
    assert infog["status"] == 0 and infop["status"] == 0
    for p, om in enumerate(oms):
        w1, w2 = rhs.draw_omegas(om, seeds[p])
        b = rhs.build_rhs(om, d=[t.cpu().numpy() for t in data[p]], omega1=w1, omega2=w2)
        ref = pcg.pcg(om.apply_A, precond.DiagonalPrecond(om), b, rtol=1e-12, maxiter=5000)
        assert ref.status == "ok"
        eg = _rel(xg[p].cpu().numpy(), ref.x)
        ep = _rel(xp[p].cpu().numpy(), ref.x)
        print(f"problem {p}: iters gpu {infog['iters'][p]} oracle {ref.iters}, err {eg:.1e} {ep:.1e}",
              flush=True)
        assert eg < SOL_TOL and ep < SOL_TOL, (p, eg, ep)
        assert abs(infog["iters"][p] - ref.iters) <= 2


_FULL = {}


def _full_batch():
    """The benchmark's batch at full size: 64 CR problems (Nside_max 64 / 128 /
    256, 1-3 components, masks) with M_diag blocks, their data and a Batch."""
    if _FULL:
        return _FULL
    torch, crsolve = _setup()
    grids = {}

    def grid(spec):
        if spec not in grids:
            grids[spec] = crsolve.Grid.from_spec(spec)
        return grids[spec]

    probs, models, data, taus_all = [], [], [], []
    for i in range(64):
        prob = inputs.make_problem("batched", index=i)
        gl = [grid(b["grid"]) for b in prob["bands"]]
        taus = inputs.inverse_noise_maps(prob, lambda spec: grid(spec).pixel_centres())
        m = crsolve.model_from_problem(prob, taus, gl, diag=True)
        s = torch.tensor(inputs.signal_coefficients(prob), device="cuda")
        sig = m.project(s)
        d = []
        for nu, (t, mp) in enumerate(zip(taus, sig)):
            tt = torch.tensor(t, device="cuda")
            rms = torch.where(tt > 0, 1.0 / torch.sqrt(torch.clamp(tt, min=1e-300)), torch.zeros_like(tt))
            z = torch.tensor(inputs.white_noise(prob, nu, len(t)), device="cuda")
            d.append((mp[0] + rms * z).contiguous())
        probs.append(prob)
        models.append(m)
        data.append(d)
        taus_all.append(taus)
        if (i + 1) % 16 == 0:
            print(f"built {i + 1}/64", flush=True)
    _FULL.update(probs=probs, models=models, data=data, taus=taus_all, grids=grids,
                 batch=crsolve.Batch(models), seeds=[p["seed"] for p in probs])
    return _FULL


@pytest.mark.timeout(900)
def test_full_size_batch_residuals():
    """The benchmark's configuration (64 full-size CR problems, M_diag, graphs,
    rtol 1e-8): every problem's true residual is within 1e-8 with the GPU's
    A, and for one problem of each Nside_max tier also with the oracle's A
    and the oracle's right-hand side (same Philox draws)."""
    print("case full-size batch residuals (bench configuration)", flush=True)
    F = _full_batch()
    xs, info = F["batch"].solve(d=F["data"], seeds=F["seeds"], mode="cr", precond="diag", rtol=1e-8,
                                maxiter=5000, use_graph=True)
    assert info["status"] == 0
    print(f"batched to 1e-8: iterations max {max(info['iters'])}", flush=True)
    for p in range(64):
        assert info["relres"][p] <= 1e-8, (p, info["relres"][p])
    for p in (0, 1, 2):  # Nside_max 64, 128, 256
        om, _ = oracle_model(F["probs"][p], F["taus"][p])
        w1, w2 = rhs.draw_omegas(om, F["seeds"][p])
        b = rhs.build_rhs(om, d=[t.cpu().numpy() for t in F["data"][p]], omega1=w1, omega2=w2)
        r = b - om.apply_A(xs[p].cpu().numpy())
        rel = float(np.linalg.norm(r) / np.linalg.norm(b))
        print(f"problem {p}: oracle residual {rel:.2e}", flush=True)
        assert rel <= 1.5e-8, (p, rel)


@pytest.mark.timeout(900)
def test_full_size_batch_matches_per_model_solves():
    """The same 64 problems solved to 1e-11 in the batch (graphs) and one by
    one: every batch solution equals its own solve to 1e-8, element by element."""
    print("case full-size batch vs per-model solves", flush=True)
    F = _full_batch()
    xs, info = F["batch"].solve(d=F["data"], seeds=F["seeds"], mode="cr", precond="diag", rtol=1e-11,
                                maxiter=8000, use_graph=True)
    assert info["status"] == 0
    worst = 0.0
    for p, m in enumerate(F["models"]):
        xr, ir = m.constrained_realization([t.unsqueeze(0) for t in F["data"][p]], F["seeds"][p],
                                           mode="cr", precond="diag", rtol=1e-11, maxiter=8000)
        assert ir["status"] == 0
        e = _rel(xs[p].cpu().numpy(), xr[0].cpu().numpy())
        worst = max(worst, e)
        assert e < SOL_TOL, (p, e)
    print(f"batch vs per-model worst max-abs rel {worst:.2e}", flush=True)
