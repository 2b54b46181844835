"""Benchmark: PCG time-to-solution per right-hand side on MI355X, batched vs plain.

Default workload "batched": 64 constrained realizations of multi-resolution
problems (Nside_max 64/128/256 in turn, bands at Nside_max x (1/4, 1/2, 1/2,
1, 1) with L_nu = 2 Nside_nu, 1-3 components, a galactic cut plus 1-degree
disks leaving sky fraction U[0.6, 0.95], lognormal noise RMS), solved to
rel.res 1e-8.  One step = one batched solve of all 64 problems from x = 0:
one stacked PCG whose iterations are captured hipGraphs, with every band of
every problem sharing the transform launches of its (grid, L).  The plain
figure solves the same 64 problems one constrained_realization call at a
time without graphs.  Under these masks the block-diagonal preconditioner is
the default; the pseudo-inverse preconditioner (which degrades under a mask)
is run on a bounded sample and its iteration count reported.  The
"multires" field is the full-sky 5-band model with pseudo-inverse vs
block-diagonal preconditioning.  All inputs are seeded, synthetic and
resident in device memory before the timed region.

Prints one JSON line, with the dominant Legendre kernel's roofline measured
live with HIP events (recorded inside the captured graphs) and the CPU
oracle's time on a bounded sample as a reported baseline.

    python bench.py [--steps K] [--warmup W] [--workload batched|multires|masked]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X published dense FP64 (vector and matrix)
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the dominant kernel family, from rocprofv3 FETCH_SIZE /
# WRITE_SIZE passes over this benchmark (scaled by a plain copy of known size);
# used only while the Legendre source is the one the counters were taken on
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "legendre_adjoint_batched_cr64_traffic.txt")
LEGENDRE_SRC = os.path.join(ROOT, "paper_1710_00621_amd", "csrc", "legendre.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(name, nprob, crsolve, inputs, torch, dev, with_mask=True):
    grids = {}

    def grid(spec):
        if spec not in grids:
            grids[spec] = crsolve.Grid.from_spec(spec)
        return grids[spec]

    probs = []
    if name == "batched":
        specs = [inputs.make_problem("batched", index=i) for i in range(nprob)]
    else:
        specs = [inputs.make_problem(name)]
    for i, prob in enumerate(specs):
        gl = [grid(b["grid"]) for b in prob["bands"]]
        taus = inputs.inverse_noise_maps(prob, lambda spec: grid(spec).pixel_centres())
        model = crsolve.model_from_problem(prob, taus, gl, diag=True)
        if with_mask and prob["mask"] is not None:
            # the mask-restricted preconditioner of M_add (setup, outside the timed region)
            mgrid, mk = crsolve.mask_of_problem(prob, taus, gl)
            model.set_mask(mgrid, mk)
        s = torch.tensor(inputs.signal_coefficients(prob), device=dev)
        sig_maps = model.project(s)
        d = []
        for nu, (t, m) in enumerate(zip(taus, sig_maps)):
            sig = torch.tensor(t, device=dev)
            sig = torch.where(sig > 0, 1.0 / torch.sqrt(torch.clamp(sig, min=1e-300)),
                              torch.zeros_like(sig))
            z = torch.tensor(inputs.white_noise(prob, nu, len(t)), device=dev)
            d.append((m + sig * z).unsqueeze(0).contiguous())
        probs.append({"prob": prob, "model": model, "d": d, "taus": taus})
        if (i + 1) % 8 == 0:
            log(f"built {i + 1}/{len(specs)} problems")
    return probs, grids


def solve_all(probs, precond, rtol, maxiter, torch, allow_notconv=False, allow=None):
    """One constrained realization per problem.  A solve that stops at maxiter
    above rtol is an error unless allow_notconv (then its status and final
    residual are kept in the problem's record); allow: the accepted statuses
    (overrides allow_notconv)."""
    iters = []
    for p in probs:
        x, info = p["model"].constrained_realization(p["d"], p["prob"]["seed"], mode=p["prob"]["rhs"],
                                                     precond=precond, rtol=rtol, maxiter=maxiter,
                                                     raise_on_error=False)
        ok = allow if allow is not None else ((0, -4) if allow_notconv else (0,))
        if info["status"] not in ok:
            raise RuntimeError(f"solve failed: status {info['status']} relres {info['relres']}")
        iters.append(info["iters"][0])
        p["x"] = x
        p["status"] = info["status"]
        p["relres"] = float(info["relres"][0])
    return iters


def sht_roofline(crsolve, torch, dev, nside=1024, lmax=2000, nmaps_list=(1, 6), reps=3):
    """Legendre kernels at the large band shape, each timed with HIP events."""
    g = crsolve.Grid.healpix(nside)
    out = {}
    for nm in nmaps_list:
        alm = torch.randn(nm, (lmax + 1) ** 2, dtype=torch.float64, device=dev)
        maps = torch.randn(nm, g.npix, dtype=torch.float64, device=dev)
        crsolve.sht_synth(g, lmax, alm)
        crsolve.sht_adjoint(g, lmax, maps)
        torch.cuda.synchronize()
        crsolve.kernel_stats_reset()
        crsolve.set_profiling(True)
        for _ in range(reps):
            crsolve.sht_synth(g, lmax, alm)
            crsolve.sht_adjoint(g, lmax, maps)
        torch.cuda.synchronize()
        crsolve.set_profiling(False)
        res = {}
        for fam in ("legendre_synth", "legendre_adjoint", "ring_fft"):
            st = crsolve.kernel_stats(fam)
            avg_ms = st["ms"] / max(1, st["launches"])
            work = st["work"] / max(1, st["launches"])
            if fam == "ring_fft":
                gbs = work / (avg_ms * 1e-3) / 1e9
                res[fam] = {"avg_ms": avg_ms, "GBs": gbs, "frac_hbm": gbs / HBM_PEAK_GBS}
            else:
                cnt = crsolve.kernel_work_counts(fam)
                n = max(1, st["launches"])
                tf = work / (avg_ms * 1e-3) / 1e12
                res[fam] = {"avg_ms": avg_ms, "TFLOPs": tf, "frac": tf / FP64_PEAK_TFLOPS,
                            "frac_nominal": cnt["nominal"] / n / (avg_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                            "frac_evaluated": cnt["evaluated"] / n / (avg_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                            "flops_per_launch": {"fp64_range": work, "nominal": cnt["nominal"] / n,
                                                 "evaluated": cnt["evaluated"] / n}}
        out[f"nside{nside}_l{lmax}_nmaps{nm}"] = res
    return out


def _oracle_model(prob, taus):
    from oracle import geometry
    from oracle.model import Model as OModel
    from paper_1710_00621_amd import inputs
    bands = [{"grid": geometry.make_grid(b["grid"]), "lmax": b["lmax"], "beam": bm, "tau": t}
             for b, bm, t in zip(prob["bands"], inputs.beams(prob), taus)]
    comps = [{"lmax": c["lmax"], "invcl": icl} for c, icl in zip(prob["comps"], inputs.priors(prob))]
    return OModel(bands, comps, prob["q"])


def _blas_threads():
    """Threads the oracle's numpy BLAS runs with (its matrix products are the
    multi-threaded part of the oracle)."""
    try:
        from threadpoolctl import threadpool_info
        n = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
        return int(n)
    except Exception:
        return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def _sht_work(prob):
    """Legendre work of one round trip over all bands: sum nring * (L+1)^2."""
    from paper_1710_00621_amd import inputs
    return sum(inputs.grid_nring(b["grid"]) * (b["lmax"] + 1) ** 2 for b in prob["bands"])


def _oracle_precond(om, precond, prob, taus):
    import numpy as np

    from oracle import mask as omask, precond as opc
    if precond == "diag":
        return opc.DiagonalPrecond(om)
    Mp = opc.PseudoInversePrecond(om)
    if precond == "pinv":
        return Mp
    nu = max(range(len(taus)), key=lambda i: len(taus[i]))
    return omask.AddPrecond(Mp, omask.MaskPrecond(om, prob["bands"][nu]["grid"][1], np.asarray(taus[nu]) == 0))


def cpu_baseline(name, probs, gpu_iters, precond, budget_s=20.0):
    """The oracle (numpy FP64, as it stands) timed on the host on a bounded
    sample, in ms per RHS.  For a single large problem the sample is one PCG
    iteration (apply_A + preconditioner) of the same recipe at reduced
    resolution (1/2; 1/8 for the 9-band masked recipe, whose half-resolution
    copy would take the oracle's naive transforms far beyond the sample
    budget), scaled by the Legendre work ratio (sum nring (L+1)^2) and
    multiplied by the GPU's iteration count."""
    import numpy as np

    from oracle import geometry, precond as opc
    from paper_1710_00621_amd import inputs

    nthreads = _blas_threads()
    if name != "batched":
        scale = {"masked": 8, "fullres": 16}.get(name, 2)
        prob = inputs.make_problem(name, scale=scale)
        cache = {}

        def centres(spec):
            if spec not in cache:
                cache[spec] = geometry.make_grid(spec).pixel_centres()
            return cache[spec]

        taus = inputs.inverse_noise_maps(prob, centres)
        om = _oracle_model(prob, taus)
        M = _oracle_precond(om, precond, prob, taus)
        v = np.random.default_rng(0).standard_normal(om.n)
        t0 = time.perf_counter()
        om.apply_A(v)
        M(v)
        dt = time.perf_counter() - t0
        ratio = _sht_work(probs[0]["prob"]) / _sht_work(prob)
        per_rhs = dt * ratio * gpu_iters[0] * 1e3
        return {"value": per_rhs, "unit": "ms/RHS", "cores": nthreads, "kind": "oracle",
                "sample": (f"one oracle PCG iteration (apply_A + M_{precond}) of the {name} recipe "
                           f"at 1/{scale} resolution took {dt:.1f} s; scaled by the Legendre work ratio "
                           f"{ratio:.2f} and by the GPU's {gpu_iters[0]} iterations (extrapolated)")}
    # batched: one problem of each Nside_max tier (the first of the tier), at
    # full resolution for the 64 and 128 tiers and at half resolution for the
    # 256 tier (scaled by the Legendre work ratio); every problem's estimate is
    # its tier's time per iteration times its own GPU iteration count
    per_iter = {}
    notes = []
    for tier_i, tier in enumerate((64, 128, 256)):
        p = probs[tier_i]
        scale = 2 if tier == 256 else 1
        prob = inputs.make_problem("batched", scale=scale, index=tier_i)
        cache = {}

        def centres(spec):
            if spec not in cache:
                cache[spec] = geometry.make_grid(spec).pixel_centres()
            return cache[spec]

        taus = p["taus"] if scale == 1 else inputs.inverse_noise_maps(prob, centres)
        om = _oracle_model(prob, taus)
        M = _oracle_precond(om, precond, prob, taus)
        v = np.random.default_rng(0).standard_normal(om.n)
        t0 = time.perf_counter()
        om.apply_A(v)
        M(v)
        dt = time.perf_counter() - t0
        ratio = _sht_work(p["prob"]) / _sht_work(prob)
        per_iter[tier] = dt * ratio
        notes.append(f"Nside_max {tier}: {dt:.2f} s at 1/{scale} resolution x {ratio:.2f}")
    est = [per_iter[(64, 128, 256)[i % 3]] * gpu_iters[i] for i in range(len(probs))]
    return {"value": 1e3 * float(np.mean(est)), "unit": "ms/RHS", "cores": nthreads, "kind": "oracle",
            "sample": ("one oracle PCG iteration (apply_A + M_" + precond + ") per Nside_max tier (" +
                       "; ".join(notes) + " by the Legendre work ratio), times each of the 64 problems' "
                       "GPU iteration counts; extrapolated per RHS")}


def _traffic(kernel, workload):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, which was taken on the batched workload: null for another
    workload or once legendre.hip has changed since the counters were read."""
    import hashlib
    if workload != "batched":
        return None
    try:
        with open(TRAFFIC_SUMMARY) as fh:
            text = fh.read()
        with open(LEGENDRE_SRC, "rb") as fh:
            sha = hashlib.sha1(fh.read()).hexdigest()
    except OSError:
        return None
    f = {}
    for line in text.splitlines():
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            f[k.strip()] = v.strip()
    if f.get("kernel") != kernel or f.get("legendre_source_sha1") != sha:
        return None
    try:
        return float(f["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _roofline(crsolve, ms_total, workload):
    """Dominant Legendre family over the timed region (the Legendre transforms
    together take the largest share of a step; the ring stage is reported
    beside them against HBM).  achieved = its flops
    counted over the (ring pair, l, m) triples whose |lambda| reaches the
    float64 range, each launch credited with the maps still active, divided
    by its summed launch time (HIP events on the launch stream, recorded in
    the captured graphs).  The nominal and the kernels' own (>= 2^-100)
    triple counts are given beside it."""
    fam = {f: crsolve.kernel_stats(f) for f in ("legendre_synth", "legendre_adjoint", "ring_fft")}
    dom = max(("legendre_synth", "legendre_adjoint"), key=lambda f: fam[f]["ms"])
    st = fam[dom]
    secs = max(1e-30, st["ms"] * 1e-3)
    achieved = st["work"] / secs / 1e12
    counts = crsolve.kernel_work_counts(dom)
    launches = max(1, st["launches"])
    ring = fam["ring_fft"]
    other = "legendre_adjoint" if dom == "legendre_synth" else "legendre_synth"
    so = fam[other]
    return {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": _traffic(dom, workload),
            "avg_launch_ms": st["ms"] / launches, "launches": st["launches"],
            "flops_per_launch": {"fp64_range": counts["fp64"] / launches,
                                 "nominal": counts["nominal"] / launches,
                                 "evaluated": counts["evaluated"] / launches},
            "frac_nominal": counts["nominal"] / secs / 1e12 / FP64_PEAK_TFLOPS,
            "frac_evaluated": counts["evaluated"] / secs / 1e12 / FP64_PEAK_TFLOPS,
            "share_of_step": st["ms"] / max(1e-9, ms_total),
            "legendre_share_of_step": (fam["legendre_synth"]["ms"] + fam["legendre_adjoint"]["ms"])
            / max(1e-9, ms_total),
            other: {"TFLOP/s": so["work"] / max(1e-30, so["ms"] * 1e-3) / 1e12,
                    "frac": so["work"] / max(1e-30, so["ms"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                    "avg_launch_ms": so["ms"] / max(1, so["launches"])},
            "ring_fft": {"GB/s": ring["work"] / max(1e-30, ring["ms"] * 1e-3) / 1e9,
                         "frac_hbm": ring["work"] / max(1e-30, ring["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "share_of_step": ring["ms"] / max(1e-9, ms_total)}}


def batch_solve(batch, probs, precond, rtol, maxiter, use_graph=True):
    d = [[t[0] for t in p["d"]] for p in probs]
    seeds = [p["prob"]["seed"] for p in probs]
    xs, info = batch.solve(d=d, seeds=seeds, mode="cr", precond=precond, rtol=rtol,
                           maxiter=maxiter, use_graph=use_graph, raise_on_error=False)
    if info["status"] != 0:
        raise RuntimeError(f"batched solve failed: status {info['status']}")
    return info["iters"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched", choices=["batched", "multires", "masked", "fullres"])
    ap.add_argument("--nprob", type=int, default=64)
    ap.add_argument("--precond", default=None, choices=["pinv", "diag", "add"])
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--maxiter", type=int, default=5000)
    ap.add_argument("--pinv-maxiter", type=int, default=3000,
                    help="batched workload: iteration cap of the reported pseudo-inverse solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sht-roofline", action="store_true")
    ap.add_argument("--no-multires", action="store_true")
    ap.add_argument("--group-streams", type=int, default=4,
                    help="also time the batch with its transform groups on this many streams (1: skip)")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched workload: skip the plain (one solve per problem) pass and the "
                         "pseudo-inverse sample")
    ap.add_argument("--sht-only", action="store_true",
                    help="time only the transforms at the large band shapes (Nside 1024 / L 2000 with "
                         "1 and 6 maps, Nside 256 / L 512 with 42 maps, Nside 2048 / L 6000) and print "
                         "them as one JSON object (for profiling runs; not the benchmark line)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a dispatch of known "
                         "traffic for scaling hardware byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X and does not shard "
              "across GPUs (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if a.precond is None:
        a.precond = {"batched": "diag", "masked": "add"}.get(a.workload, "pinv")
    if a.workload != "batched":
        a.nprob = 1

    import torch

    from paper_1710_00621_amd import crsolve, inputs

    dev = torch.device("cuda:0")
    if a.copy_probe_mb > 0:
        nel = a.copy_probe_mb * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)  # one elementwise kernel: reads and writes copy_probe_mb MiB
        torch.cuda.synchronize()
        del src, dst
    if a.sht_only:
        res = sht_roofline(crsolve, torch, dev)
        res.update(sht_roofline(crsolve, torch, dev, nside=256, lmax=512, nmaps_list=(42,)))
        res.update(sht_roofline(crsolve, torch, dev, nside=2048, lmax=6000, nmaps_list=(1,), reps=2))
        print(json.dumps({"sht_roofline": res}), flush=True)
        return
    t0 = time.time()
    free0 = torch.cuda.mem_get_info(dev)[0]
    # the mask hierarchies (M_add) only where a solve uses them
    need_mask = a.precond == "add" or a.workload == "masked" or (a.workload == "batched" and not a.no_plain)
    probs, grids = build_workload(a.workload, a.nprob, crsolve, inputs, torch, dev, with_mask=need_mask)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    log(f"setup {setup_s:.1f}s for {len(probs)} problems")
    nrhs = len(probs)
    extra = {}

    if a.workload == "batched":
        tb = time.time()
        batch = crsolve.Batch([p["model"] for p in probs])
        setup_s += time.time() - tb
        for w in range(a.warmup):
            it = batch_solve(batch, probs, a.precond, a.rtol, a.maxiter)
            log(f"warmup {w}: batched iterations max {max(it)}")
            if not a.no_plain:
                solve_all(probs, a.precond, a.rtol, a.maxiter, torch)
        torch.cuda.synchronize()
        crsolve.kernel_stats_reset()
        crsolve.set_profiling(True)
        t1 = time.perf_counter()
        for k in range(a.steps):
            iters = batch_solve(batch, probs, a.precond, a.rtol, a.maxiter)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        crsolve.set_profiling(False)
        ms_per_step = (t2 - t1) * 1e3 / a.steps
        per_rhs = ms_per_step / nrhs
        roof = _roofline(crsolve, ms_per_step * a.steps, a.workload)
        log(f"batched: {ms_per_step:.1f} ms/step, {per_rhs:.3f} ms/RHS")
        gstats = batch.stats()
        extra["graphs"] = {**gstats, "iterations_per_launch": gstats["iterations"] / max(1, gstats["graph_launches"])}
        if a.group_streams > 1:
            # the same solves with the transform groups on several streams
            # (outside the timed region, no profiling: concurrent kernels'
            # event durations overlap, so the roofline above is taken with
            # the groups serialized)
            batch.set_streams(a.group_streams)
            batch_solve(batch, probs, a.precond, a.rtol, a.maxiter)
            torch.cuda.synchronize()
            tc = time.perf_counter()
            for k in range(a.steps):
                batch_solve(batch, probs, a.precond, a.rtol, a.maxiter)
            torch.cuda.synchronize()
            conc_rhs = (time.perf_counter() - tc) * 1e3 / a.steps / nrhs
            batch.set_streams(1)
            log(f"batched, groups on {a.group_streams} streams: {conc_rhs:.3f} ms/RHS")
            extra["concurrent_groups"] = {"streams": a.group_streams, "ms_per_RHS": conc_rhs,
                                          "speedup": per_rhs / conc_rhs}
        mode = (f"batched: one stacked PCG over all {nrhs} problems in chunks of 8 iterations per "
                f"captured hipGraph launch (convergence tested on the device, the host reading flags "
                f"between chunks; finished transform groups left out)")
        # Legendre kernel variant per (grid, L) group, as picked by the autotuner at batch creation
        groups = {}
        for p in probs:
            for b in p["prob"]["bands"]:
                key = (b["grid"], b["lmax"])
                groups[key] = groups.get(key, 0) + 1
        extra["legendre_autotuned"] = {
            f"{spec[0]} {spec[1]} L{L} x{n} maps": crsolve.legendre_choice(grids[spec], L, n)
            for (spec, L), n in sorted(groups.items(), key=lambda kv: kv[0][1])}
    if a.workload == "batched" and not a.no_plain:
        # plain: the same problems one constrained_realization call at a time, no graphs
        torch.cuda.synchronize()
        tp = time.perf_counter()
        it_p = solve_all(probs, a.precond, a.rtol, a.maxiter, torch)
        torch.cuda.synchronize()
        plain_rhs = (time.perf_counter() - tp) * 1e3 / nrhs
        log(f"plain: {plain_rhs:.3f} ms/RHS")
        mode += f"; plain = {nrhs} separate constrained_realization calls without graphs"
        extra["plain_ms_per_rhs"] = plain_rhs
        extra["speedup_batched_over_plain"] = plain_rhs / per_rhs
        extra["plain_iterations_sum"] = int(sum(it_p))
        # the same batch with the pseudo-inverse preconditioner (the paper's
        # preconditioner; it degrades under masks), one solve, bounded
        if a.precond != "pinv":
            torch.cuda.synchronize()
            tq = time.perf_counter()
            d = [[t[0] for t in p["d"]] for p in probs]
            xs_pi, info_pi = batch.solve(d=d, seeds=[p["prob"]["seed"] for p in probs], mode="cr",
                                         precond="pinv", rtol=a.rtol, maxiter=a.pinv_maxiter,
                                         use_graph=True, raise_on_error=False)
            torch.cuda.synchronize()
            t_pi = (time.perf_counter() - tq) * 1e3
            extra["batched_pinv"] = {
                "ms_per_rhs": t_pi / nrhs, "status": info_pi["status"],
                "converged": info_pi["status"] == 0, "iterations_max": max(info_pi["iters"]),
                "iterations_mean": sum(info_pi["iters"]) / nrhs,
                "relres_max": max(info_pi["relres"]), "maxiter": a.pinv_maxiter,
                "note": "M_PI on the same masked batch (tau^+ = 0 in the mask); a time to solution "
                        "only when converged"}
            log(f"batched pinv: {extra['batched_pinv']}")
        # the mask-restricted M_add on every problem, one solve each (plain)
        if a.precond != "add":
            torch.cuda.synchronize()
            ta = time.perf_counter()
            # M_add (J taken as I in the V-cycle) is not symmetric positive definite in
            # general: a solve may stop on r . z <= 0 (CRS_EBREAKDOWN, status -5); such
            # problems are counted, not raised
            it_a = solve_all(probs, "add", a.rtol, a.maxiter, torch, allow=(0, -4, -5))
            torch.cuda.synchronize()
            st = [p["status"] for p in probs]
            conv = [i for i, s_ in zip(it_a, st) if s_ == 0]
            extra["plain_add"] = {
                "ms_per_rhs": (time.perf_counter() - ta) * 1e3 / nrhs,
                "converged": len(conv), "breakdown": st.count(-5), "not_converged": st.count(-4),
                "breakdown_problems": [{"problem": i, "iterations": it_a[i], "relres": probs[i]["relres"]}
                                       for i in range(nrhs) if st[i] == -5],
                "iterations_max": max(conv) if conv else None,
                "iterations_mean": sum(conv) / len(conv) if conv else None,
                "iterations_sum": int(sum(it_a)),
                "note": "M_add = M_PI + M_mask (multigrid V-cycle on the mask), one constrained_realization "
                        "per problem without graphs; compare plain_ms_per_rhs / plain_iterations_sum (M_diag)"}
            log(f"plain add: {extra['plain_add']}")
        # the pseudo-inverse preconditioner on the smallest problem (bounded)
        if a.precond != "pinv":
            small = min(probs, key=lambda p: p["model"].n)
            tq = time.perf_counter()
            x, info = small["model"].constrained_realization(
                small["d"], small["prob"]["seed"], mode="cr", precond="pinv", rtol=a.rtol,
                maxiter=3000, raise_on_error=False)
            torch.cuda.synchronize()
            extra["pinv_sample"] = {
                "problem_n": small["model"].n, "status": info["status"], "iters": info["iters"][0],
                "relres": info["relres"][0], "ms": (time.perf_counter() - tq) * 1e3,
                "note": "pseudo-inverse preconditioner under a mask (tau^+ = 0 there), maxiter 3000"}
            log(f"pinv sample: {extra['pinv_sample']}")
    elif a.workload != "batched":
        if a.workload == "fullres":
            # memory plan of the single large model: tables and operator state,
            # against the device memory the run actually took
            mb, eb = probs[0]["model"].plan_bytes(1)
            extra["memory"] = {"model_tables_GiB": mb / 2 ** 30, "operator_state_GiB": eb / 2 ** 30}
        # the masked workload may stop at maxiter above rtol (reported, not an error)
        nc = a.workload == "masked"
        for w in range(a.warmup):
            it = solve_all(probs, a.precond, a.rtol, a.maxiter, torch, allow_notconv=nc)
            log(f"warmup {w}: iterations {it}")
        torch.cuda.synchronize()
        crsolve.kernel_stats_reset()
        crsolve.set_profiling(True)
        t1 = time.perf_counter()
        for k in range(a.steps):
            iters = solve_all(probs, a.precond, a.rtol, a.maxiter, torch, allow_notconv=nc)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        crsolve.set_profiling(False)
        ms_per_step = (t2 - t1) * 1e3 / a.steps
        per_rhs = ms_per_step / nrhs
        roof = _roofline(crsolve, ms_per_step * a.steps, a.workload)
        mode = "plain (one right-hand side per solve)"
        if any(p["status"] != 0 for p in probs):
            # not a time-to-solution: the time of maxiter iterations
            extra["converged"] = False
            extra["final_relres"] = [p["relres"] for p in probs]
            extra["ms_per_iteration"] = ms_per_step / max(1, sum(iters))
            log(f"not converged to {a.rtol} in {a.maxiter} iterations: relres {extra['final_relres']}")
        log(f"timed {a.steps} steps: {ms_per_step:.1f} ms/step, {per_rhs:.3f} ms/RHS")
        if a.workload == "fullres":
            torch.cuda.synchronize()
            extra["memory"]["device_used_GiB"] = (free0 - torch.cuda.mem_get_info(dev)[0]) / 2 ** 30
            extra["memory"]["device_total_GiB"] = torch.cuda.mem_get_info(dev)[1] / 2 ** 30
            log(f"memory: {extra['memory']}")
        if a.workload == "masked":
            # the other preconditioners for five times as many iterations (they
            # do not reach rtol under the mask): residual reached and time per iteration
            comp = {}
            for pc in [p_ for p_ in ("diag", "pinv") if p_ != a.precond]:
                cap = 5 * max(iters)
                torch.cuda.synchronize()
                tc = time.perf_counter()
                itc = solve_all(probs, pc, a.rtol, cap, torch, allow_notconv=True)
                torch.cuda.synchronize()
                dtc = (time.perf_counter() - tc) * 1e3
                comp[pc] = {"iterations": itc[0], "converged": probs[0]["status"] == 0,
                            "relres": probs[0]["relres"], "ms_per_iteration": dtc / max(1, itc[0])}
                log(f"masked with {pc}: {comp[pc]}")
            extra["preconditioner_comparison"] = comp

    if a.workload != "multires" and not a.no_multires:
        mp, _ = build_workload("multires", 1, crsolve, inputs, torch, dev)
        res = {}
        for pc in ("pinv", "diag"):
            solve_all(mp, pc, a.rtol, a.maxiter, torch)
            torch.cuda.synchronize()
            tm = time.perf_counter()
            itm = solve_all(mp, pc, a.rtol, a.maxiter, torch)
            torch.cuda.synchronize()
            res[pc] = {"ms_per_rhs": (time.perf_counter() - tm) * 1e3, "iterations": itm[0]}
        res["speedup_pinv_over_diag"] = res["diag"]["ms_per_rhs"] / res["pinv"]["ms_per_rhs"]
        extra["multires"] = res
        log(f"multires: {res}")
    elif a.workload == "multires":
        other = "diag" if a.precond == "pinv" else "pinv"
        tc = time.perf_counter()
        it_o = solve_all(probs, other, a.rtol, a.maxiter, torch)
        torch.cuda.synchronize()
        t_o = (time.perf_counter() - tc) * 1e3 / len(probs)
        extra["preconditioner_comparison"] = {"precond": other, "ms_per_rhs": t_o,
                                              "iterations_mean": sum(it_o) / len(it_o)}

    out = {
        "metric": "PCG time-to-solution/RHS at rel.res 1e-8, batched vs plain; SHT % roofline",
        "value": per_rhs, "unit": "ms/RHS", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": a.workload, "problems": nrhs, "precond": a.precond,
                   "rtol": a.rtol, "mode": mode, "setup_s": setup_s,
                   "iterations": {"min": min(iters), "mean": sum(iters) / len(iters),
                                  "max": max(iters)}, **extra},
        "roofline": roof,
    }
    if not a.no_sht_roofline:
        out["sht_roofline"] = sht_roofline(crsolve, torch, dev)
        # full resolution: Nside 2048 (8192-pixel rings), L = 6000
        out["sht_roofline"].update(sht_roofline(crsolve, torch, dev, nside=2048, lmax=6000, nmaps_list=(1,), reps=2))
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.workload, probs, iters, a.precond)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
