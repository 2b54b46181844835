"""torch.autograd Functions over the library (argument marshalling only; every
transform and solve runs in the HIP library).

SHTSynth / SHTAdjoint: y = Y a and a = Y^T f; each one's backward is the
other transform (Y and Y^T are exact adjoints, Sect. 2.1 / Sect. 3.2).

WienerSolve: x = A(q)^-1 b(q, d) with A = S^-1 + sum_nu P_nu^T N_nu^-1 P_nu and
b = sum_nu P_nu^T N_nu^-1 d_nu (Sect. 2.3), P_nu = Y_nu B_nu q_{nu,k}.  The
backward is one more PCG solve with the symmetric A (implicit function
theorem): lam = A^-1 g, dL/db = lam, dL/dd_nu = N^-1 P_nu lam and
dL/dq = lam^T (db/dq - (dA/dq) x)  (apply_db_dmix, apply_dA_dmix).

PriorQuad: 1/2 x^T S^-1 x.  Chi2: sum_nu (d_nu - P_nu x)^T N_nu^-1 (d_nu - P_nu x),
with dChi2/dq_{nu,k} = -2 x_k . [B Y^T N^-1 (d - P x)]_nu (apply_db_dmix).

mixing_matrix: q_{nu,k}(beta) for CMB / power-law / modified-black-body
components, written with torch so that dq/dbeta comes from autograd.
"""
import math

import torch

from . import crsolve
from ._lib import check, lib, PRECOND

H_OVER_K = 0.04799243  # h / k_B in K / GHz


class SHTSynth(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alm, grid, lmax):
        ctx.grid, ctx.lmax = grid, lmax
        return crsolve.sht_synth(grid, lmax, alm.contiguous())

    @staticmethod
    def backward(ctx, gmap):
        return crsolve.sht_adjoint(ctx.grid, ctx.lmax, gmap.contiguous()), None, None


class SHTAdjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, maps, grid, lmax):
        ctx.grid, ctx.lmax = grid, lmax
        return crsolve.sht_adjoint(grid, lmax, maps.contiguous())

    @staticmethod
    def backward(ctx, galm):
        return crsolve.sht_synth(ctx.grid, ctx.lmax, galm.contiguous()), None, None


def sht_synth(alm, grid, lmax):
    return SHTSynth.apply(alm, grid, lmax)


def sht_adjoint(maps, grid, lmax):
    return SHTAdjoint.apply(maps, grid, lmax)


def _vecptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


def _band_array(model, maps):
    import ctypes
    arr = (ctypes.c_void_p * model.nbands)()
    keep = []
    for i, t in enumerate(maps):
        if t is None:
            arr[i] = None
        else:
            t = t.contiguous()
            keep.append(t)
            arr[i] = t.data_ptr()
    return arr, keep


def dA_dmix(model, lam, x):
    """-lam^T (dA/dq) x as a [nbands, ncomp] tensor (one right-hand side)."""
    dq = torch.empty((model.nbands, model.ncomp), dtype=torch.float64, device=x.device)
    check(lib().apply_dA_dmix(model._h, 1, _vecptr(lam.contiguous()), _vecptr(x.contiguous()),
                              _vecptr(dq), crsolve._stream(x.device)))
    return dq


def db_dmix(model, lam, maps):
    """lam^T (db/dq) for b = sum P^T N^-1 maps, as a [nbands, ncomp] tensor."""
    dq = torch.empty((model.nbands, model.ncomp), dtype=torch.float64, device=lam.device)
    arr, keep = _band_array(model, maps)
    check(lib().apply_db_dmix(model._h, 1, _vecptr(lam.contiguous()), arr, _vecptr(dq),
                              crsolve._stream(lam.device)))
    return dq


def prior_inv(model, x):
    y = torch.empty_like(x)
    check(lib().apply_prior_inv(model._h, 1, _vecptr(x.contiguous()), _vecptr(y),
                                crsolve._stream(x.device)))
    return y


class _Mixing:
    """Sets the model's mixing matrix to q for the duration of a block and
    puts the previous one back (a backward pass may run after other forwards
    have set another q on the same model)."""

    def __init__(self, model, q):
        self.model, self.q = model, q.detach().cpu().numpy()

    def __enter__(self):
        self.prev = getattr(self.model, "_q_now", None)
        if self.prev is None or not (self.prev.shape == self.q.shape and (self.prev == self.q).all()):
            self.model.set_mixing(self.q)
            self.model._q_now = self.q
        return self

    def __exit__(self, *exc):
        if self.prev is not None and self.model._q_now is not self.prev:
            self.model.set_mixing(self.prev)
            self.model._q_now = self.prev
        return False


class WienerSolve(torch.autograd.Function):
    """x = A(q)^-1 sum_nu P_nu^T N_nu^-1 d_nu; d given as per-band [npix] tensors."""

    @staticmethod
    def forward(ctx, q, model, opts, *d):
        qd = q.detach()
        with _Mixing(model, qd):
            b = model.build_rhs(d=[t.detach().unsqueeze(0) for t in d])[0]
            x, info = model.pcg(b, precond=opts.get("precond", "pinv"), rtol=opts.get("rtol", 1e-12),
                                maxiter=opts.get("maxiter", 5000))
        ctx.model, ctx.opts, ctx.qdev = model, opts, q.device
        ctx.save_for_backward(qd, x, *[t.detach() for t in d])
        return x

    @staticmethod
    def backward(ctx, gx):
        q, x, *d = ctx.saved_tensors
        model, opts = ctx.model, ctx.opts
        with _Mixing(model, q):
            lam, _ = model.pcg(gx.contiguous(), precond=opts.get("precond", "pinv"),
                               rtol=opts.get("rtol", 1e-12), maxiter=opts.get("maxiter", 5000))
            grad_q = db_dmix(model, lam, d) + dA_dmix(model, lam, x)
            # dL/dd_nu = N^-1 P_nu lam
            grad_d = model.noise_weight(model.project(lam))
        return (grad_q.to(ctx.qdev), None, None, *grad_d)


class PriorQuad(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, model):
        val, y = model.prior_quad(x.detach())
        ctx.save_for_backward(y)
        return val

    @staticmethod
    def backward(ctx, g):
        (y,) = ctx.saved_tensors
        return g * y, None


class Chi2(torch.autograd.Function):
    """sum_nu (d_nu - P_nu x)^T N_nu^-1 (d_nu - P_nu x) at mixing q."""

    @staticmethod
    def forward(ctx, x, q, model, *d):
        qd = q.detach()
        with _Mixing(model, qd):
            val, res = model.chi2(x.detach(), [t.detach() for t in d])
        ctx.model, ctx.qdev = model, q.device
        ctx.save_for_backward(qd, x.detach(), *res)
        return val

    @staticmethod
    def backward(ctx, g):
        q, x, *res = ctx.saved_tensors
        model = ctx.model
        with _Mixing(model, q):
            # dChi2/dx = -2 sum P^T N^-1 r ; dChi2/dq = -2 x_k . [B Y^T N^-1 r] ; dChi2/dd = 2 N^-1 r
            grad_x = g * model.build_rhs(d=[r.unsqueeze(0) for r in res])[0]
            grad_q = db_dmix(model, x, res)
            wres = model.noise_weight(res, scale=2.0)
        return -2.0 * grad_x, (-2.0 * g * grad_q).to(ctx.qdev), None, *[g * w for w in wres]


def mixing_matrix(freqs, comps, beta):
    """q[nu, k] for components given as dicts with kind in {cmb, sync, dust},
    nu_ref and T (dust); beta: tensor with one entry per component (ignored
    for CMB)."""
    rows = []
    for f in freqs:
        row = []
        for k, c in enumerate(comps):
            if c["kind"] == "cmb":
                row.append(torch.ones((), dtype=torch.float64, device=beta.device))
            elif c["kind"] == "sync":
                row.append((f / c["nu_ref"]) ** beta[k])
            else:
                T = c.get("T", 20.0)
                x = H_OVER_K * f / T
                x0 = H_OVER_K * c["nu_ref"] / T
                row.append((f / c["nu_ref"]) ** (beta[k] + 1.0) * (math.expm1(x0) / math.expm1(x)))
        rows.append(torch.stack(row))
    return torch.stack(rows)


def wf_loss(model, d, q, opts=None):
    """L = 1/2 x^T S^-1 x + chi^2 at the Wiener filter x(q, d)."""
    opts = opts or {}
    x = WienerSolve.apply(q, model, opts, *d)
    return PriorQuad.apply(x, model) + Chi2.apply(x, q, model, *d), x
