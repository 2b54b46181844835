"""Preconditioned conjugate gradients (oracle).  TEST INFRASTRUCTURE ONLY.

Sect. 2.3: A is symmetric positive definite, so CG is the solver; it starts
from x_1 = 0 (or a given x0), uses the residual r = b - A x as the error
proxy, and a symmetric positive definite preconditioner M.  The iteration
is the standard Hestenes-Stiefel form (the tutorial the paper cites):

    r = b - A x;  z = M r;  p = z;  rho = r.z
    repeat:  q = A p;  a = rho / p.q;  x += a p;  r -= a q
             stop if |r| / |b| <= rtol   (recursive residual)
             z = M r;  rho' = r.z;  p = z + (rho'/rho) p;  rho = rho'

When the recursive residual passes, the true residual b - A x is formed
once; if it fails the tolerance the iteration restarts from the current x.
Breakdown (p.q <= 0, r.z <= 0 or a non-finite scalar) is reported.
"""
import numpy as np


class PCGResult:
    def __init__(self, x, iters, relres, status, history, errors):
        self.x = x
        self.iters = iters
        self.relres = relres
        self.status = status  # "ok", "maxiter", "breakdown"
        self.history = history  # recursive |r|/|b| after each iteration
        self.errors = errors    # |x_i - x_true| / |x_true| when x_true given
        self.iterates = []


def pcg(apply_A, apply_M, b, x0=None, rtol=1e-8, maxiter=1000, x_true=None,
        keep_iterates=0):
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.sqrt(b @ b))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    hist, errs, iterates = [], [], []
    if bnorm == 0.0:
        res = PCGResult(np.zeros_like(b), 0, 0.0, "ok", hist, errs)
        return res
    r = b - apply_A(x) if x0 is not None else b.copy()
    z = apply_M(r)
    p = z.copy()
    rho = float(r @ z)
    if not np.isfinite(rho) or rho <= 0.0:
        return PCGResult(x, 0, float(np.sqrt(r @ r)) / bnorm, "breakdown", hist, errs)
    status = "maxiter"
    it = 0
    while it < maxiter:
        it += 1
        q = apply_A(p)
        pq = float(p @ q)
        if not np.isfinite(pq) or pq <= 0.0:
            status = "breakdown"
            break
        a = rho / pq
        x = x + a * p
        r = r - a * q
        rel = float(np.sqrt(r @ r)) / bnorm
        hist.append(rel)
        if x_true is not None:
            errs.append(float(np.linalg.norm(x - x_true) / np.linalg.norm(x_true)))
        if len(iterates) < keep_iterates:
            iterates.append(x.copy())
        if not np.isfinite(rel):
            status = "breakdown"
            break
        if rel <= rtol:
            rt = b - apply_A(x)
            if float(np.sqrt(rt @ rt)) / bnorm <= rtol:
                status = "ok"
                break
            r = rt  # restart from the current iterate
            z = apply_M(r)
            p = z.copy()
            rho = float(r @ z)
            continue
        z = apply_M(r)
        rho_new = float(r @ z)
        if not np.isfinite(rho_new) or rho_new <= 0.0:
            status = "breakdown"
            break
        p = z + (rho_new / rho) * p
        rho = rho_new
    rt = b - apply_A(x)
    res = PCGResult(x, it, float(np.sqrt(rt @ rt)) / bnorm, status, hist, errs)
    res.iterates = iterates
    return res
