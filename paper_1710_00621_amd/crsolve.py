"""Python binding of the crsolve C ABI on torch tensors.

Every operation runs in the HIP library; this module only checks tensor
shapes, device and dtype, passes raw pointers and the current torch stream,
and turns status codes into exceptions.  Tensors are float64, contiguous and
on a CUDA (HIP) device.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

c_double_p = _lib.c_double_p


def _stream(dev=None):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _dev_f64(t, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU device")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _host_f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(c_double_p)


def nalm(lmax):
    return (lmax + 1) * (lmax + 1)


class Grid:
    """HEALPix RING or Gauss-Legendre ring grid (library handle)."""

    def __init__(self, handle):
        self._h = handle
        nr = ctypes.c_int()
        npix = ctypes.c_int64()
        check(lib().crs_grid_info(self._h, ctypes.byref(nr), ctypes.byref(npix)))
        self.nring = nr.value
        self.npix = npix.value

    @classmethod
    def healpix(cls, nside):
        h = ctypes.c_void_p()
        check(lib().crs_grid_healpix(int(nside), ctypes.byref(h)))
        g = cls(h)
        g.spec = ("healpix", int(nside))
        return g

    @classmethod
    def gauss_legendre(cls, nrings, nphi):
        h = ctypes.c_void_p()
        check(lib().crs_grid_gauss_legendre(int(nrings), int(nphi), ctypes.byref(h)))
        g = cls(h)
        g.spec = ("gl", int(nrings), int(nphi))
        return g

    @classmethod
    def from_spec(cls, spec):
        if spec[0] == "healpix":
            return cls.healpix(spec[1])
        if spec[0] == "gl":
            return cls.gauss_legendre(spec[1], spec[2])
        raise ValueError(spec)

    def pixel_centres(self):
        z = np.empty(self.npix)
        phi = np.empty(self.npix)
        check(lib().crs_grid_pixel_centres(self._h, z.ctypes.data_as(c_double_p),
                                           phi.ctypes.data_as(c_double_p)))
        return z, phi

    def reserve(self, lmax, nmaps, device=None):
        """Build the (grid, lmax) tables and the transform workspace for up to
        nmaps maps, so later sht_synth / sht_adjoint calls allocate nothing."""
        check(lib().crs_sht_reserve(self._h, int(lmax), int(nmaps), _stream(device)))

    def weights(self):
        w = np.empty(self.npix)
        check(lib().crs_grid_weights(self._h, w.ctypes.data_as(c_double_p)))
        return w

    def close(self):
        if getattr(self, "_h", None):
            lib().crs_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _as2d(t):
    return (t.unsqueeze(0), True) if t.dim() == 1 else (t, False)


def sht_synth(grid, lmax, alm, out=None):
    """Y alm (Sect. 2.1): alm [nmaps, (lmax+1)^2] or [(lmax+1)^2] -> maps."""
    a, sq = _as2d(alm)
    if a.shape[1] != nalm(lmax):
        raise ValueError("alm has the wrong length for lmax")
    nm = a.shape[0]
    if out is None:
        out = torch.empty((nm, grid.npix), dtype=torch.float64, device=a.device)
    o2, _ = _as2d(out)
    check(lib().sht_synth(grid._h, int(lmax), nm, _dev_f64(a, "alm"), a.stride(0),
                          _dev_f64(o2, "out"), o2.stride(0), _stream(a.device)))
    return out[0] if (sq and out.dim() == 2) else out


def autotune_legendre(grid, lmax, nmaps, device=None):
    """Time every Legendre kernel variant for (grid, lmax, nmaps) and keep the
    fastest synthesis and adjoint for later transforms of that shape."""
    dev = torch.device("cuda") if device is None else torch.device(device)
    check(lib().crs_autotune_legendre(grid._h, int(lmax), int(nmaps), _stream(dev)))
    return legendre_choice(grid, lmax, nmaps)


def legendre_choice(grid, lmax, nmaps):
    """The Legendre kernel variant in use for a shape: dict with synth_mfma,
    synth_pairs_per_lane, adjoint_mfma, adjoint_pairs_per_lane,
    adjoint_tiles_per_wave."""
    out = (ctypes.c_int * 5)()
    check(lib().crs_legendre_choice(grid._h, int(lmax), int(nmaps), out))
    keys = ("synth_mfma", "synth_pairs_per_lane", "adjoint_mfma", "adjoint_pairs_per_lane",
            "adjoint_tiles_per_wave")
    return dict(zip(keys, list(out)))


def sht_adjoint(grid, lmax, maps, out=None):
    """Y^T maps (adjoint synthesis, Sect. 3.2)."""
    m, sq = _as2d(maps)
    if m.shape[1] != grid.npix:
        raise ValueError("map has the wrong number of pixels")
    nm = m.shape[0]
    if out is None:
        out = torch.empty((nm, nalm(lmax)), dtype=torch.float64, device=m.device)
    o2, _ = _as2d(out)
    check(lib().sht_adjoint(grid._h, int(lmax), nm, _dev_f64(m, "maps"), m.stride(0),
                            _dev_f64(o2, "out"), o2.stride(0), _stream(m.device)))
    return out[0] if (sq and out.dim() == 2) else out


class Model:
    """Model handle: bands (grid, L_nu, beam, tau, q row) and components
    (L_k, C_k^-1).  ``diag`` also builds the M_diag blocks."""

    def __init__(self, bands, comps, q, diag=True):
        self.grids = [b["grid"] for b in bands]
        self.taus = [np.asarray(b["tau"], dtype=np.float64) for b in bands]
        self.ncomp = len(comps)
        self.nbands = len(bands)
        self.lmax_comp = [int(c["lmax"]) for c in comps]
        self.band_lmax = [int(b["lmax"]) for b in bands]
        q = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(self.nbands, self.ncomp))
        keep = []
        bd = (_lib.BandDesc * self.nbands)()
        for i, b in enumerate(bands):
            beam, pb = _host_f64(b["beam"])
            tau, pt = _host_f64(b["tau"])
            qr, pq = _host_f64(q[i])
            if len(tau) != b["grid"].npix:
                raise ValueError("tau has the wrong length")
            if len(beam) < b["lmax"] + 1:
                raise ValueError("beam shorter than lmax + 1")
            keep += [beam, tau, qr]
            bd[i] = _lib.BandDesc(b["grid"]._h, int(b["lmax"]), pb, pt, pq)
        lk = (ctypes.c_int * self.ncomp)(*self.lmax_comp)
        icl = (c_double_p * self.ncomp)()
        for k, c in enumerate(comps):
            a, p = _host_f64(c["invcl"])
            if len(a) < c["lmax"] + 1:
                raise ValueError("invcl shorter than lmax + 1")
            keep.append(a)
            icl[k] = p
        desc = _lib.ModelDesc(self.ncomp, lk, icl, self.nbands, bd, 1 if diag else 0)
        h = ctypes.c_void_p()
        check(lib().crs_model_create(ctypes.byref(desc), _stream(), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int64()
        check(lib().crs_model_size(self._h, ctypes.byref(n)))
        self.n = n.value
        self.has_diag = bool(diag)

    def close(self):
        if getattr(self, "_h", None):
            lib().crs_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def plan_bytes(self, nrhs=1):
        """(model tables, operator state for nrhs right-hand sides) in bytes."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        check(lib().crs_model_plan_bytes(self._h, int(nrhs), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def alpha2(self):
        a = np.empty(self.nbands)
        check(lib().crs_model_alpha2(self._h, a.ctypes.data_as(c_double_p)))
        return a

    def set_mixing(self, q):
        q, p = _host_f64(np.asarray(q, dtype=np.float64).reshape(self.nbands, self.ncomp))
        check(lib().crs_model_set_mixing(self._h, p, _stream()))

    def set_mixing_map(self, band, comp, grid=None, qmap=None):
        """Spatially varying mixing for (band, comp): Q~ = Y^T W diag(qmap) Y on
        grid (eq:Q); qmap None returns the pair to its scalar q."""
        if qmap is None:
            check(lib().crs_model_set_mixing_map(self._h, int(band), int(comp), None, None, _stream()))
            return
        q, p = _host_f64(qmap)
        if len(q) != grid.npix:
            raise ValueError("qmap must have one value per pixel of grid")
        check(lib().crs_model_set_mixing_map(self._h, int(band), int(comp), grid._h, p, _stream()))
        self._mixgrids = getattr(self, "_mixgrids", []) + [grid]

    def merge_observations(self, groups):
        """Merge bands in the pseudo-inverse preconditioner (App. A.3):
        groups is a list of lists of band indices (None or [] clears)."""
        if not groups:
            check(lib().crs_model_merge_observations(self._h, None, _stream()))
            return
        g = [-1] * self.nbands
        for gi, grp in enumerate(groups):
            for nu in grp:
                g[nu] = gi
        arr = (ctypes.c_int * self.nbands)(*g)
        check(lib().crs_model_merge_observations(self._h, arr, _stream()))

    def set_mask(self, grid, mask, lowpass_r2=0.0, omega=0.0, nbottom=0, rcond=0.0, exact_j=False):
        """Build the mask-restricted preconditioner (M_mask; CRS_PRECOND_ADD =
        M_PI + M_mask) on a HEALPix grid; mask: bool / uint8 per pixel (True =
        masked).  Zero option values select the defaults; exact_j applies
        J = Y^T W Y exactly in the cycle (symmetric V-cycle)."""
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        if m.shape != (grid.npix,):
            raise ValueError("mask must have one entry per pixel of the grid")
        opts = _lib.MaskOpts(float(lowpass_r2), float(omega), int(nbottom), float(rcond), 1 if exact_j else 0)
        check(lib().crs_model_set_mask(self._h, grid._h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                       ctypes.byref(opts), _stream()))
        self.mask_grid = grid

    def mask_info(self):
        """[(Nside, L, masked pixels)] per level of the mask multigrid."""
        nl = ctypes.c_int()
        out = (ctypes.c_int * 96)()
        check(lib().crs_model_mask_info(self._h, ctypes.byref(nl), out, 96))
        return [tuple(out[3 * h:3 * h + 3]) for h in range(min(nl.value, 32))]

    def apply_mask(self, r):
        return self._op(lib().apply_mask_precond, r, "r")

    def _vec(self, x, name):
        x2, sq = _as2d(x)
        if x2.shape[1] != self.n:
            raise ValueError(f"{name} must have n = {self.n} entries per right-hand side")
        return x2, sq

    def _op(self, fn, x, name):
        x2, sq = self._vec(x, name)
        y = torch.empty_like(x2)
        check(fn(self._h, x2.shape[0], _dev_f64(x2, name), _dev_f64(y, "out"), _stream(x2.device)))
        return y[0] if sq else y

    def apply_A(self, x):
        return self._op(lib().apply_A, x, "x")

    def apply_pinv(self, r):
        return self._op(lib().apply_pinv_precond, r, "r")

    def apply_diag(self, r):
        return self._op(lib().apply_diag_precond, r, "r")

    def pcg(self, b, precond="pinv", rtol=1e-8, maxiter=1000, x0=None, history=False,
            raise_on_error=True):
        b2, sq = self._vec(b, "b")
        nrhs = b2.shape[0]
        x = torch.zeros_like(b2) if x0 is None else self._vec(x0, "x0")[0].clone()
        iters = (ctypes.c_int * nrhs)()
        rel = (ctypes.c_double * nrhs)()
        hist = np.zeros((max(1, maxiter), nrhs)) if history else None
        hp = hist.ctypes.data_as(c_double_p) if history else None
        st = lib().pcg_solve(self._h, _lib.PRECOND[precond], nrhs, _dev_f64(b2, "b"),
                             _dev_f64(x, "x"), float(rtol), int(maxiter), iters, rel, hp,
                             _stream(b2.device))
        if raise_on_error:
            check(st)
        info = {"status": st, "iters": list(iters), "relres": list(rel)}
        if history:
            info["history"] = hist[:max(info["iters"] + [0])]
        return (x[0] if sq else x), info

    def build_rhs(self, d=None, omega1=None, omega2=None, nrhs=1):
        dev = torch.device("cuda")
        keep = []

        def ptrs(lst):
            if lst is None:
                return None
            arr = (ctypes.c_void_p * self.nbands)()
            for i, t in enumerate(lst):
                if t is None:
                    arr[i] = None
                else:
                    t = t.contiguous()
                    keep.append(t)
                    arr[i] = _dev_f64(t, "map")
            return arr

        b = torch.empty((nrhs, self.n), dtype=torch.float64, device=dev)
        w2 = None
        if omega2 is not None:
            w2t = omega2.contiguous()
            keep.append(w2t)
            w2 = _dev_f64(w2t, "omega2")
        check(lib().build_rhs(self._h, nrhs, ptrs(d), ptrs(omega1), w2, _dev_f64(b, "b"),
                              _stream(dev)))
        return b

    def _maps_arg(self, maps, keep):
        """Host array of per-band device pointers (None entries stay NULL)."""
        if maps is None:
            return None
        arr = (ctypes.c_void_p * self.nbands)()
        for i, t in enumerate(maps):
            if t is None:
                arr[i] = None
            else:
                t = t.contiguous()
                keep.append(t)
                arr[i] = _dev_f64(t, "map")
        return arr

    def prior_quad(self, x):
        """(1/2 x^T S^-1 x per right-hand side [nrhs], S^-1 x)."""
        x2, sq = self._vec(x, "x")
        y = torch.empty_like(x2)
        val = torch.empty(x2.shape[0], dtype=torch.float64, device=x2.device)
        check(lib().crs_prior_quad(self._h, x2.shape[0], _dev_f64(x2, "x"), _dev_f64(y, "y"),
                                   _dev_f64(val, "val"), _stream(x2.device)))
        return (val[0], y[0]) if sq else (val, y)

    def chi2(self, x, d):
        """(chi^2 = sum_nu (d - P x)^T N^-1 (d - P x) per right-hand side,
        residual maps d - P x as a list of [nrhs, npix_nu] tensors).  d: per
        band [nrhs, npix_nu] (or [npix_nu]) tensors, None = zero."""
        x2, sq = self._vec(x, "x")
        nrhs = x2.shape[0]
        keep = []
        dd = None if d is None else [None if t is None else (t.unsqueeze(0) if t.dim() == 1 else t)
                                     for t in d]
        res = [torch.empty((nrhs, g.npix), dtype=torch.float64, device=x2.device) for g in self.grids]
        rarr = (ctypes.c_void_p * self.nbands)(*[r.data_ptr() for r in res])
        val = torch.empty(nrhs, dtype=torch.float64, device=x2.device)
        check(lib().crs_chi2(self._h, nrhs, _dev_f64(x2, "x"), self._maps_arg(dd, keep), rarr,
                             _dev_f64(val, "val"), _stream(x2.device)))
        return (val[0], [r[0] for r in res]) if sq else (val, res)

    def noise_weight(self, maps, scale=1.0):
        """scale N_nu^-1 maps_nu for every band (list of [nrhs, npix_nu] or [npix_nu])."""
        keep = []
        sq = maps[0].dim() == 1
        mm = [t.unsqueeze(0) if t.dim() == 1 else t for t in maps]
        nrhs = mm[0].shape[0]
        out = [torch.empty((nrhs, g.npix), dtype=torch.float64, device=mm[0].device) for g in self.grids]
        oarr = (ctypes.c_void_p * self.nbands)(*[o.data_ptr() for o in out])
        check(lib().crs_noise_weight(self._h, nrhs, float(scale), self._maps_arg(mm, keep), oarr,
                                     _stream(mm[0].device)))
        return [o[0] for o in out] if sq else out

    def project(self, x):
        """P_nu x for every band: list of [nrhs, npix_nu] tensors."""
        x2, sq = self._vec(x, "x")
        nrhs = x2.shape[0]
        outs = [torch.empty((nrhs, g.npix), dtype=torch.float64, device=x2.device)
                for g in self.grids]
        arr = (ctypes.c_void_p * self.nbands)(*[o.data_ptr() for o in outs])
        check(lib().crs_model_project(self._h, nrhs, _dev_f64(x2, "x"), arr, _stream(x2.device)))
        return [o[0] for o in outs] if sq else outs

    def constrained_realization(self, d, seed, mode="cr", precond="pinv", rtol=1e-8,
                                maxiter=1000, nrhs=1, raise_on_error=True):
        dev = torch.device("cuda")
        keep = []
        arr = None
        if d is not None:
            arr = (ctypes.c_void_p * self.nbands)()
            for i, t in enumerate(d):
                t = t.contiguous()
                keep.append(t)
                arr[i] = _dev_f64(t, "d")
        x = torch.empty((nrhs, self.n), dtype=torch.float64, device=dev)
        iters = (ctypes.c_int * nrhs)()
        rel = (ctypes.c_double * nrhs)()
        st = lib().constrained_realization(self._h, nrhs, arr, ctypes.c_uint64(seed), _lib.MODE[mode],
                                           _lib.PRECOND[precond], float(rtol), int(maxiter),
                                           _dev_f64(x, "x"), iters, rel, _stream(dev))
        if raise_on_error:
            check(st)
        return x, {"status": st, "iters": list(iters), "relres": list(rel)}


class Batch:
    """Many models solved together (one stacked PCG, shared transform
    launches).  The models must stay alive while the batch exists."""

    def __init__(self, models):
        self.models = list(models)
        arr = (ctypes.c_void_p * len(self.models))(*[m._h.value for m in self.models])
        h = ctypes.c_void_p()
        check(lib().crs_batch_create(arr, len(self.models), _stream(), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().crs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, d=None, seeds=None, mode="cr", precond="pinv", rtol=1e-8, maxiter=1000,
              use_graph=True, raise_on_error=True):
        """d: None or per problem None / list of per-band [npix] device tensors.
        Returns (list of [n_p] solutions, info)."""
        dev = torch.device("cuda")
        npb = len(self.models)
        keep = []
        darr = None
        if d is not None:
            darr = (ctypes.POINTER(ctypes.c_void_p) * npb)()
            for p, dl in enumerate(d):
                if dl is None:
                    darr[p] = None
                    continue
                a = (ctypes.c_void_p * self.models[p].nbands)()
                for i, t in enumerate(dl):
                    if t is None:
                        a[i] = None
                    else:
                        t = t.contiguous()
                        keep.append(t)
                        a[i] = _dev_f64(t, "d")
                keep.append(a)
                darr[p] = ctypes.cast(a, ctypes.POINTER(ctypes.c_void_p))
        sarr = None
        if seeds is not None:
            sarr = (ctypes.c_uint64 * npb)(*[int(v) for v in seeds])
        xs = [torch.empty(m.n, dtype=torch.float64, device=dev) for m in self.models]
        xarr = (ctypes.c_void_p * npb)(*[x.data_ptr() for x in xs])
        iters = (ctypes.c_int * npb)()
        rel = (ctypes.c_double * npb)()
        st = lib().crs_batch_solve(self._h, _lib.MODE[mode], darr, sarr, _lib.PRECOND[precond],
                                   float(rtol), int(maxiter), xarr, iters, rel,
                                   1 if use_graph else 0, _stream(dev))
        if raise_on_error:
            check(st)
        return xs, {"status": st, "iters": list(iters), "relres": list(rel)}

    def set_streams(self, n):
        """Run the transform groups on up to n HIP streams (1..8)."""
        check(lib().crs_batch_set_streams(self._h, int(n)))

    def stats(self):
        """Counters of the last solve: iterations, graph_launches,
        graph_captures, host_syncs."""
        out = (ctypes.c_int * 4)()
        check(lib().crs_batch_stats(self._h, out))
        return dict(zip(("iterations", "graph_launches", "graph_captures", "host_syncs"), list(out)))


def philox_normals(seed, stream, rhs, n, device="cuda"):
    out = torch.empty(n, dtype=torch.float64, device=device)
    check(lib().crs_philox_normals(ctypes.c_uint64(seed), ctypes.c_uint64(stream),
                                   ctypes.c_uint64(rhs), int(n), _dev_f64(out, "out"),
                                   _stream(out.device)))
    return out


def set_profiling(on):
    check(lib().crs_set_profiling(1 if on else 0))


def kernel_stats(family):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    w = ctypes.c_double()
    check(lib().crs_kernel_stats(family.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(w)))
    return {"launches": n.value, "ms": ms.value, "work": w.value}


def kernel_work_counts(family):
    """Summed work of a kernel family three ways: float64-range triples
    (the headline count), nominal triples, evaluated (>= 2^-100) triples."""
    out = (ctypes.c_double * 3)()
    check(lib().crs_kernel_work_counts(family.encode(), out))
    return {"fp64": out[0], "nominal": out[1], "evaluated": out[2]}


def kernel_stats_reset():
    check(lib().crs_kernel_stats_reset())


def mask_of_problem(problem, taus, grids):
    """(grid, mask) for the mask preconditioner: the finest band's HEALPix grid
    and its masked pixels (tau = 0)."""
    nu = max(range(len(taus)), key=lambda i: len(taus[i]))
    return grids[nu], np.asarray(taus[nu]) == 0.0


def model_from_problem(problem, taus, grids=None, diag=True):
    """Library model for a recipe from ``inputs`` with given tau maps."""
    from . import inputs
    if grids is None:
        cache = {}
        grids = []
        for b in problem["bands"]:
            if b["grid"] not in cache:
                cache[b["grid"]] = Grid.from_spec(b["grid"])
            grids.append(cache[b["grid"]])
    beams = inputs.beams(problem)
    bands = [{"grid": g, "lmax": b["lmax"], "beam": bm, "tau": t}
             for g, b, bm, t in zip(grids, problem["bands"], beams, taus)]
    comps = [{"lmax": c["lmax"], "invcl": icl}
             for c, icl in zip(problem["comps"], inputs.priors(problem))]
    return Model(bands, comps, problem["q"], diag=diag)
