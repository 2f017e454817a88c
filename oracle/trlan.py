"""Algorithms 1 (TRLAN-JSYM) and 2 (LANCZOS_JSYM) of the paper, FP64 NumPy.

Test infrastructure only (see the package docstring).

The steps follow the paper's order and notation (Sec. 3, Algorithms 1 and 2)
with 0-based indices: V has columns v_0..v_m, the projected matrix Tbar is
(m+1) x m and real.  Readings taken where the paper is silent or inconsistent:

* The Lanczos vector is normalised by the norm measured after the last
  reorthogonalisation pass (b1), and t_{j+1,j} = b1.  As printed, Alg. 2 divides
  by b0, which at loop exit is the norm before the last pass.
* t_{jj} = v_j^H (A v_j) is complex in floating point: the complex value is
  subtracted, its real part enters T (alpha is real, Sec. 2).
* is_convd is cleared at the start of every convergence check (Alg. 1 never
  resets it, which would leave stale flags after re-sorting).
* Sorting is stable: ascending Ritz values for the lowest end, descending for
  the largest end; the converged-first partition keeps the desired order.
* Breakdown: if the new Lanczos norm is <= breakdown_factor * u * max|T|
  (u: the unit roundoff of the storage precision), the Krylov space is
  invariant.  The reorthogonalisation loop stops there too (as printed it
  never exits when the new vector lies in the span, e.g. once the J-half
  Krylov space is exhausted at m = n/2, Sec. 2).  The cycle then ends at that
  dimension, the coupling to v_{m+1}
  is zero, and every candidate's true residual is checked; if not all nev
  pairs converge the solve stops with status "breakdown".
* tol is absolute as in the paper; tol_relative=True scales it by the largest
  |Ritz value| seen so far, a running maximum over the cycles (an estimate of
  ||A||_2 that never shrinks).  A per-cycle scale would move with the window's
  extreme Ritz value, and a pair decoupled as converged is frozen, so a pair
  whose residual sits at the threshold could drop out of the converged set
  and never return.
* min_passes > 1 takes the sqrt(2) test only from that pass on (default 1,
  the paper's rule).
* The J-restriction uses w_i = J v_i^* (Alg. 2 builds W alongside V).  With
  jsym=False the W-projections are dropped, giving the standard TRLAN that the
  paper compares against (Sec. 3).
* Invert mode (Alg. 1 and 2, invert branches): the Lanczos steps take
  u = A^-1 v_j from the caller's solve(); the Ritz values theta of T are those
  of A^-1, and the wanted end of A's spectrum is the opposite end of theta's
  (the lowest eigenvalues of a positive definite A are the largest theta), so
  the sort is reversed.  ev = 1/theta, res_est = c |t_{m+1,i} ev_i| with
  c = ||A v_{m+1}||, and the true residual uses A itself.  Every solve counts
  as one matvec in n_mv (Sec. 3); the application of A for c is counted in
  n_resid_mv with the true-residual checks.  After a breakdown there is no
  v_{m+1} and c = 0 (the couplings are zero anyway).  With tol_relative the
  scale is the running maximum of c and of the wanted |ev_i|, both lower
  bounds on ||A||_2 as max |theta| is in normal mode.
"""
from __future__ import annotations

import math
import time

import numpy as np

from .jsym import J_apply


def _w(v):
    """w = J v^* (Alg. 2 constructs W this way)."""
    return J_apply(np.conj(v))


def lanczos_jsym(apply, V, T, k, m, stats, jsym=True, breakdown_tol_fn=None, trace=None,
                 min_passes=1):
    """Algorithm 2: extend the decomposition from dimension k to m.

    apply(v) is A v in normal mode and A^-1 v in invert mode.
    V: (n, m+1) complex128 with v_0..v_k valid; T: (m+1, m) real with rows
    0..k valid.  Returns the dimension actually reached (m, or less on
    breakdown) and the breakdown flag.
    """
    gamma = math.sqrt(2.0)                       # reorthogonalisation threshold
    for j in range(k, m):
        u = apply(V[:, j])                       # A v_j, or A^-1 v_j (invert mode)
        stats["n_mv"] += 1
        t = np.vdot(V[:, j], u)                  # t_jj = v_j^H v_{j+1}
        T[j, j] = t.real
        u = u - V[:, j] * t
        b0 = np.linalg.norm(u)
        tolb = breakdown_tol_fn(T, j) if breakdown_tol_fn is not None else 0.0
        stats["_p"] = 0
        while True:                              # iterated Gram-Schmidt
            for i in range(j + 1):
                if jsym:
                    w = _w(V[:, i])
                    c = np.vdot(w, u)            # orthogonalise to W_j
                    u = u - w * c
                c = np.vdot(V[:, i], u)          # orthogonalise to V_j
                u = u - V[:, i] * c
            b1 = np.linalg.norm(u)
            stats["gs_passes"] += 1
            passes = stats.setdefault("_p", 0) + 1
            stats["_p"] = passes
            if (passes >= min_passes and b1 * gamma > b0) or b1 <= tolb:
                break
            b0 = b1
        if trace is not None and len(trace["alpha"]) < trace["cap"]:
            trace["alpha"].append(float(t.real))
            trace["beta"].append(float(b1))
        if b1 <= tolb:
            T[j + 1, j] = 0.0
            return j + 1, True
        V[:, j + 1] = u / b1
        T[j + 1, j] = b1
    return m, False


def _sym_T(T, m):
    """The m x m symmetric projected matrix from the lower entries of Tbar."""
    Tm = np.tril(T[:m, :m])
    return Tm + np.tril(Tm, -1).T


def trlan_jsym(apply, n, nev, mwin, m, tol, which="lowest", v1=None,
               max_cycles=100000, jsym=True, unit_roundoff=2.0 ** -53,
               breakdown_factor=64.0, trace_cap=0, record_history=False,
               time_limit=None, on_cycle=None, min_passes=1, tol_relative=False,
               mode="normal", solve=None):
    """Algorithm 1: thick-restart Lanczos for a Hermitian J-symmetric A.

    apply(v) -> A v; in mode "invert" also solve(v) -> A^-1 v, which drives
    the Lanczos steps.  Returns a dict with ev (nev, desired order), X (n, nev),
    res (true residual norms), and counters n_mv (Lanczos matvecs only, as in
    Sec. 3), n_conv (outer iterations), gs_passes, n_resid_mv, status
    ("ok", "not_converged", "breakdown", "time_limit").
    on_cycle(V, T, k), if given, sees the shrunk decomposition after every
    restart (columns 0..k of V, rows 0..k of T).
    """
    if n % 2 or nev < 1 or not (nev <= mwin < m) or (jsym and m > n // 2) or m > n:
        raise ValueError("invalid parameters")
    if mode not in ("normal", "invert") or (mode == "invert" and solve is None):
        raise ValueError("mode must be 'normal' or 'invert' (the latter with solve)")
    invert = mode == "invert"
    step = solve if invert else apply
    # sort key on theta: the wanted end of A's spectrum, reversed under inversion
    descending = (which == "lowest") == invert
    stats = dict(n_mv=0, gs_passes=0, n_resid_mv=0, n_conv=0)
    trace = dict(alpha=[], beta=[], cap=trace_cap) if trace_cap else None
    history = []
    V = np.zeros((n, m + 1), dtype=np.complex128)
    T = np.zeros((m + 1, m))
    v = np.ones(n, dtype=np.complex128) if v1 is None else np.asarray(v1, dtype=np.complex128).copy()
    V[:, 0] = v / np.linalg.norm(v)             # initial unit vector
    k = 0
    t0 = time.perf_counter()

    def btol(Tb, j):
        return breakdown_factor * unit_roundoff * max(np.abs(Tb[:j + 2, :j + 1]).max(), 1e-300)

    status = "not_converged"
    ev = res = None
    icnv = 0
    scale = 0.0                                  # running max |theta| (tol_relative)
    for cycle in range(max_cycles):
        stats["n_conv"] += 1
        meff, broke = lanczos_jsym(step, V, T, k, m, stats, jsym=jsym,
                                   breakdown_tol_fn=btol, trace=trace, min_passes=min_passes)
        if meff < nev:                           # invariant subspace too small
            status = "breakdown"
            ev = np.full(nev, np.nan)
            res = np.full(nev, np.inf)
            icnv = 0
            break
        Tm = _sym_T(T, meff)
        lam, Z = np.linalg.eigh(Tm)              # T_m = Z Lambda Z^T
        order = np.argsort(-lam if descending else lam, kind="stable")
        lam = lam[order]
        Z = Z[:, order]
        V[:, :meff] = V[:, :meff] @ Z            # V_m := V_m Z_m
        s = T[meff, meff - 1] * Z[meff - 1, :]   # t_{m+1,i} = t_{m+1,m} z_{m,i}
        if invert:
            ev = 1.0 / lam[:nev]                 # ev(i) = 1/lambda_i
            c = 0.0
            if not broke:
                c = np.linalg.norm(apply(V[:, meff]))   # c = ||A v_{m+1}||
                stats["n_resid_mv"] += 1
            res_est = c * np.abs(s[:nev] * ev)
            scale = max(scale, c, np.abs(ev).max())
        else:
            ev = lam[:nev].copy()
            res_est = np.abs(s[:nev])
            scale = max(scale, np.abs(lam).max())
        res = np.full(nev, np.inf)
        is_convd = np.zeros(nev, dtype=bool)
        tol_c = tol * scale if tol_relative else tol
        for i in range(nev):
            if res_est[i] < tol_c:               # check true residuals
                r = apply(V[:, i]) - V[:, i] * ev[i]
                stats["n_resid_mv"] += 1
                res[i] = np.linalg.norm(r)
                is_convd[i] = res[i] < tol_c
        # converged first, desired order kept (stable partition)
        perm = np.concatenate([np.flatnonzero(is_convd), np.flatnonzero(~is_convd),
                               np.arange(nev, meff)]).astype(int)
        lam = lam[perm]
        s = s[perm]
        V[:, :meff] = V[:, perm]
        ev = ev[perm[:nev]]
        res = res[perm[:nev]]
        res_est = res_est[perm[:nev]]
        icnv = int(is_convd.sum())
        s[:icnv] = 0.0                           # decouple converged subspace
        if record_history:
            history.append(dict(k=k, meff=meff, icnv=icnv, ev=ev.copy(), res_est=res_est.copy()))
        if icnv == nev:
            status = "ok"
            break
        if broke:
            status = "breakdown"
            break
        if time_limit is not None and time.perf_counter() - t0 > time_limit:
            status = "time_limit"
            break
        k = min(icnv + mwin, m - 1)              # shrink (eq. dynamicwin)
        T[:] = 0.0
        T[np.arange(k), np.arange(k)] = lam[:k]
        T[k, :k] = s[:k]
        V[:, k] = V[:, meff]
        if on_cycle is not None:
            on_cycle(V, T, k)
    stats.pop("_p", None)
    out = dict(ev=ev, X=V[:, :nev].copy(), res=res, status=status, icnv=icnv,
               history=history, **stats)
    if trace is not None:
        out["alpha"] = np.array(trace["alpha"])
        out["beta"] = np.array(trace["beta"])
    return out
