"""Conjugate gradients for the invert mode (Sec. 4.2: A^-1 v by CG), FP64.

Test infrastructure only (see the package docstring).

The textbook method of Hestenes and Stiefel for a Hermitian positive definite
A (complex inner products, x_0 = 0):

    r_0 = b, p_0 = r_0
    alpha_k = (r_k^H r_k) / (p_k^H A p_k)
    x_{k+1} = x_k + alpha_k p_k
    r_{k+1} = r_k - alpha_k A p_k
    beta_k  = (r_{k+1}^H r_{k+1}) / (r_k^H r_k)
    p_{k+1} = r_{k+1} + beta_k p_k

stopping when the recursive residual satisfies ||r_k|| <= rtol ||b||.  The
paper names the method but fixes neither the start nor the stopping rule;
x_0 = 0 and the relative recursive-residual test are the readings taken here.
"""
from __future__ import annotations

import numpy as np


def cg(apply, b, rtol, maxit):
    """Solve A x = b.  Returns (x, iterations, converged, history of ||r_k||)."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.vdot(r, r).real
    bnorm = np.sqrt(rr)
    hist = [bnorm]
    if bnorm == 0.0:
        return x, 0, True, hist
    it = 0
    while it < maxit and np.sqrt(rr) > rtol * bnorm:
        q = apply(p)
        pq = np.vdot(p, q).real          # p^H A p is real for Hermitian A
        alpha = rr / pq
        x = x + alpha * p
        r = r - alpha * q
        rr_new = np.vdot(r, r).real
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        it += 1
        hist.append(np.sqrt(rr))
    return x, it, bool(np.sqrt(rr) <= rtol * bnorm), hist
