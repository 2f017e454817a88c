#!/usr/bin/env python3
"""Benchmark of the J-symmetric thick-restart Lanczos solver on one MI355X.

The default workload is the 32^4 J-stencil (n = 8388608, 200 lowest pairs,
m = 500, mwin = 250).  For the stencil workloads a step is one outer
iteration of Algorithm 1 (the Lanczos steps of Algorithm 2 with their
J-restricted reorthogonalisation, the Rayleigh-Ritz step, the basis update
and the true-residual checks): one mixed-precision solve (FP32 complex
operator and basis, FP64 reductions and Ritz problem) runs to the nev
converged pairs, its first W iterations are the warm-up and the next K are
timed (the solver records the wall time at the end of every iteration, where
the device is idle); `value` is the wall time of that whole solve, i.e. the
mixed time to the nev converged pairs.  The plain FP64 solver runs the same
W + K iterations on the same input, so the two precisions are compared on
the same steps.  For the other workloads a step is one complete solve (or
one replay of the batched graph).

    python bench.py [--steps K] [--warmup W]
                    [--workload stencil32|stencil16|dense4096|batched512|casea|invert16|
                                tek289|tek289inv]

Prints one JSON line.  Only one GPU is used; --gpus N > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to k converged eigenpairs (mixed vs FP64, same GPU); matvec HBM GB/s"
HBM_PEAK_GBPS = 8000.0
# per-kernel HIP events in the iteration-step solves at every 8th Lanczos step
# (the operator applies and Gram-Schmidt kernels of the other steps run
# without events between them)
TIMING_STRIDE = 8

WORKLOADS = {
    # 4D J-stencil, d = 4, Haar links, complex normal B (seeded)
    "stencil16": dict(kind="stencil", L=(16, 16, 16, 16), seed=4, nev=100, m=300, mwin=150,
                      tol=1e-5, tol_relative=False, step="cycle"),
    "stencil32": dict(kind="stencil", L=(32, 32, 32, 32), seed=5, nev=200, m=500, mwin=250,
                      tol=1e-5, tol_relative=False, step="cycle"),
    # dense random Hermitian J-symmetric, n = 4096; the mixed tolerance is
    # relative to max|theta| (the FP32 matvec itself errs by ~2e-5 here)
    "dense4096": dict(kind="dense", h=2048, seed=2, nev=50, m=160, mwin=80, tol=1e-5,
                      tol_relative=True, tol_fp64=1e-10),
    # 512 dense problems, even n uniform in 64..1024, one persistent launch
    # replayed from a hipGraph; tolerance relative to max|theta| in both forms
    "batched512": dict(kind="batched", seed=3, count=512, nev=8, m=32, mwin=16, tol=1e-5,
                       tol_relative=True, tol_fp64=1e-10),
    # invert mode (A^-1 v_j by conjugate gradients) on the 16^4 J-stencil,
    # which is positive definite; the paper's small-eigenvalue parameters
    # for TRLAN-JSYM (nev, mwin, m) = (8, 16, 48)
    "invert16": dict(kind="stencil", L=(16, 16, 16, 16), seed=4, nev=8, m=48, mwin=16,
                     tol=1e-5, tol_relative=False, invert=True, cg_tol=1e-7),
    # Case B operator (Sec. 4.2): A = D D^H, twisted Eguchi-Kawai Wilson-Dirac
    # with Haar SU(289) links in place of the Monte Carlo ensemble (n = 334080,
    # the paper's size); the paper's (nev, mwin, m) = (8, 16, 48) for the large
    # eigenvalues in normal mode and the small ones in invert mode
    "tek289": dict(kind="tek", N=289, kappa=0.15, seed=289, nev=8, m=48, mwin=16,
                   which="largest", tol=1e-5, tol_relative=True, tol_fp64=1e-10),
    "tek289inv": dict(kind="tek", N=289, kappa=0.15, seed=289, nev=8, m=48, mwin=16,
                      which="lowest", tol=1e-5, tol_relative=True, tol_fp64=1e-10,
                      invert=True, cg_tol=1e-6, cg_tol_fp64=1e-11),
    # Table 1 (Case A, Sec. 4.1): ten known-spectrum matrices of size 2000,
    # largest eigenvalues, tol 1e-13, FP64; the J-restricted method against
    # the standard one over the published (nev, mwin, m) grid
    "casea": dict(kind="casea", n=2000, seeds=list(range(8, 18)), tol=1e-13),
}


def describe(w):
    if w["kind"] == "casea":
        return (f"Case A: {len(w['seeds'])} known-spectrum Hermitian J-symmetric matrices, n={w['n']}, "
                f"largest eigenvalues, tol={w['tol']:g}, FP64, seeds {w['seeds'][0]}..{w['seeds'][-1]}; "
                "TRLAN-JSYM and standard TRLAN over the Table 1 grid")
    if w["kind"] == "batched":
        return (f"batched: {w['count']} dense Hermitian J-symmetric problems, even n uniform in "
                f"64..1024, {w['nev']} lowest pairs each, m={w['m']}, mwin={w['mwin']}, "
                f"tol={w['tol']:g} rel (mixed) / {w['tol_fp64']:g} rel (fp64), seed {w['seed']}, "
                f"one persistent launch in a hipGraph")
    if w["kind"] == "tek":
        N = w["N"]
        inv = (f", invert mode (CG to {w['cg_tol']:g} / {w['cg_tol_fp64']:g})" if w.get("invert")
               else ", normal mode")
        return (f"Case B operator A = D D^H (twisted Eguchi-Kawai Wilson-Dirac, J = C gamma_5), "
                f"N={N} (n={4 * (N * N - 1)}), kappa={w['kappa']}, Haar SU(N) links seed {w['seed']}, "
                f"{w['nev']} {w['which']} pairs, m={w['m']}, mwin={w['mwin']}, tol={w['tol']:g} rel "
                f"(mixed) / {w['tol_fp64']:g} rel (fp64){inv}")
    if w["kind"] == "stencil":
        L = w["L"]
        n = 2 * int(np.prod(L)) * 4
        inv = (f", invert mode (CG to {w['cg_tol']:g})" if w.get("invert") else "")
        return (f"4D J-stencil {'x'.join(map(str, L))} d=4 (n={n}), {w['nev']} lowest pairs, "
                f"m={w['m']}, mwin={w['mwin']}, tol={w['tol']:g} abs, seed {w['seed']}{inv}")
    n = 2 * w["h"]
    return (f"dense Hermitian J-symmetric n={n}, {w['nev']} lowest pairs, m={w['m']}, "
            f"mwin={w['mwin']}, tol={w['tol']:g} rel (mixed) / {w['tol_fp64']:g} abs (fp64), "
            f"seed {w['seed']}")


def _known_spectrum_blocks(seed, n):
    from threadpoolctl import threadpool_limits
    from paper_2001_07428_amd import inputs
    with threadpool_limits(1):   # one BLAS thread per worker process
        return inputs.known_spectrum(seed, n)[:3]


def make_host_inputs(w):
    from paper_2001_07428_amd import inputs
    if w["kind"] == "casea":   # ~17 s per matrix of size 2000: one process each
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=min(len(w["seeds"]), os.cpu_count() or 1, 16)) as ex:
            mats = list(ex.map(_known_spectrum_blocks, w["seeds"], [w["n"]] * len(w["seeds"])))
        return dict(mats=mats)
    if w["kind"] == "batched":
        n, probs = inputs.batched_dense(w["seed"], count=w["count"])
        return dict(n=n, probs=probs)
    if w["kind"] == "stencil":
        U, B = inputs.stencil_links(w["seed"], w["L"])
        return dict(U=U, B=B)
    if w["kind"] == "tek":
        return dict(U=inputs.haar_su(w["seed"], w["N"], 4))
    A11, A12 = inputs.dense_jsym(w["seed"], w["h"])
    return dict(A11=A11, A12=A12)


def make_op(J, ctx, w, host, dtype):
    import torch
    if w["kind"] == "stencil":
        U = torch.from_numpy(host["U"]).to("cuda:0", dtype)
        B = torch.from_numpy(host["B"]).to("cuda:0", dtype)
        return J.jl_op_create_stencil(ctx, w["L"], U, B)
    if w["kind"] == "tek":
        return J.jl_op_create_tek(ctx, torch.from_numpy(host["U"]).to("cuda:0", dtype), w["kappa"])
    A11 = torch.from_numpy(host["A11"]).to("cuda:0", dtype)
    A12 = torch.from_numpy(host["A12"]).to("cuda:0", dtype)
    return J.jl_op_create_dense(ctx, A11, A12)


def cycle_step_time(ct, warmup, steps):
    """Mean wall time of outer iterations warmup+1 .. warmup+steps, from the
    times ct[c] at the end of iteration c+1 (measured from the solve's start)."""
    if steps < 1 or len(ct) < warmup + steps:
        raise RuntimeError(f"the solve took {len(ct)} outer iterations, fewer than warmup + steps = "
                           f"{warmup + steps}: lower --steps/--warmup")
    start = ct[warmup - 1] if warmup > 0 else 0.0
    return (ct[warmup + steps - 1] - start) / steps


def run_cycles(J, ctx, w, host, mixed, steps, warmup, verbose, full):
    """One event-timed solve with the wall time of every outer iteration.
    full: run to the nev converged pairs (else stop after warmup + steps
    iterations).  Returns the solve's wall time, the time per iteration over
    iterations warmup+1 .. warmup+steps, and the solve's statistics."""
    import torch
    dtype = torch.complex64 if mixed else torch.complex128
    op = make_op(J, ctx, w, host, dtype)
    tol = w["tol"]
    nb = J.jl_workspace_bytes(op, w["nev"], w["m"], w["mwin"], tol)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    # loads the code objects and touches the workspace (a 4-step solve)
    J.jl_solve(op, 2, 8, 4, tol, max_cycles=1, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = J.jl_solve(op, w["nev"], w["m"], w["mwin"], tol, timing=TIMING_STRIDE, workspace=ws,
                     verbose=verbose, max_cycles=0 if full else warmup + steps,
                     cycle_times_cap=100000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ct = out.cycle_times
    if full and out.status != J.JL_OK:
        raise RuntimeError(f"solve did not converge: status {out.status}, stats {out.stats}")
    res = dict(wall=wall, step=cycle_step_time(ct, warmup, steps), stats=dict(out.stats), last=out,
               n=op.n, cycle_times=ct)
    del ws, op
    torch.cuda.empty_cache()
    return res


def run_precision(J, ctx, w, host, mixed, steps, warmup, verbose):
    import torch
    dtype = torch.complex64 if mixed else torch.complex128
    op = make_op(J, ctx, w, host, dtype)
    tol = w["tol"] if mixed or "tol_fp64" not in w else w["tol_fp64"]
    inv = bool(w.get("invert", False))
    nb = J.jl_workspace_bytes(op, w["nev"], w["m"], w["mwin"], tol, invert=inv)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda:0")

    cg_tol = w.get("cg_tol", 0.0) if mixed else w.get("cg_tol_fp64", w.get("cg_tol", 0.0))
    rel = w["tol_relative"] if (mixed or w["kind"] == "tek") else False

    def solve(timing):
        return J.jl_solve(op, w["nev"], w["m"], w["mwin"], tol, which=w.get("which", "lowest"),
                          tol_relative=rel, timing=timing, workspace=ws, verbose=verbose,
                          invert=inv, cg_tol=cg_tol)

    for _ in range(warmup):
        solve(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [solve(False) for _ in range(steps)]   # the timed steps carry no event timing
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timed = solve(True)                           # one more solve for the per-kernel breakdown
    for o in outs + [timed]:
        if o.status != J.JL_OK:
            raise RuntimeError(f"solve did not converge: status {o.status}, stats {o.stats}")
    # --steps 0 (for shapes whose solves take minutes): the event-timed solve
    # alone, its wall time as the step time
    sec = (t1 - t0) / steps if steps else timed.stats["t_total"]
    res = dict(seconds=sec, stats=dict(timed.stats), last=outs[-1] if outs else timed, n=op.n)
    del ws, op
    torch.cuda.empty_cache()
    return res


def run_batched(J, ctx, w, host, mixed, steps, warmup):
    """Timed replays of the batched graph; a step solves all problems."""
    import torch
    dtype = torch.complex64 if mixed else torch.complex128
    A11s = [torch.from_numpy(a).to("cuda:0", dtype) for a, _ in host["probs"]]
    A12s = [torch.from_numpy(c).to("cuda:0", dtype) for _, c in host["probs"]]
    tol = w["tol"] if mixed else w["tol_fp64"]
    b = J.Batch(ctx, A11s, A12s, w["nev"], w["m"], w["mwin"], tol, tol_relative=w["tol_relative"])
    for _ in range(warmup):
        b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [b.run() for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc, ev, res, st, stats = outs[-1]
    if rc != J.JL_OK:
        raise RuntimeError(f"batched solve: {(st != 0).sum()} problems did not converge")
    shape, tuned = b.shape, b.tuned
    n = host["n"].astype(np.float64)
    es = 8 if mixed else 16
    # algorithmic operator bytes: [A11 A12] (es * n^2 / 2) per Lanczos matvec
    mv_bytes = float((stats["n_mv"] * es * n * n / 2).sum())
    res_bytes = float((stats["n_resid"] * es * n * n / 2).sum())   # residual-check applies
    sec = (t1 - t0) / steps
    out = dict(seconds=sec, n_mv_total=int(stats["n_mv"].sum()),
               n_resid_total=int(stats["n_resid"].sum()), cycles_max=int(stats["cycles"].max()),
               gs_passes_total=int(stats["gs_passes"].sum()), res_max_rel=float(
                   (res / np.maximum(np.abs(ev).max(axis=1, keepdims=True), 1.0)).max()),
               matvec_bytes=mv_bytes, resid_apply_bytes=res_bytes, evals=ev, shape=shape,
               tuned_shape=tuned)
    # workgroup time per phase, summed over the problems (device wall clock)
    phases = ("apply", "gs", "ritz", "restart", "resid")
    tot = {ph: float(stats["t_" + ph].sum()) for ph in phases}
    allt = sum(tot.values())
    out["phase_seconds"] = {ph: round(v, 6) for ph, v in tot.items()}
    out["phase_share"] = {ph: round(v / allt, 4) if allt > 0 else None for ph, v in tot.items()}
    # the problem whose solve ends last sets the launch's critical path
    per = sum(stats["t_" + ph] for ph in phases)
    out["longest_problem_seconds"] = float(per.max())
    del b, A11s, A12s
    torch.cuda.empty_cache()
    return out


def main_batched(args, J, ctx, w, host):
    mixed = run_batched(J, ctx, w, host, True, args.steps, args.warmup)
    line = dict(metric=METRIC, value=round(mixed["seconds"], 5), unit="s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=round(mixed["seconds"] * 1e3, 3),
                higher_is_better=False, scaling="weak", vs_baseline=None, dtype="fp32+fp64",
                data="synthetic",
                config=dict(workload=describe(w), name=args.workload, count=w["count"], nev=w["nev"],
                            m=w["m"], mwin=w["mwin"], parallelism="1 GPU"))
    gbps = mixed["matvec_bytes"] / mixed["seconds"] / 1e9
    op_bytes = mixed["matvec_bytes"] + mixed["resid_apply_bytes"]
    op_gbps = op_bytes / mixed["seconds"] / 1e9
    line["mixed"] = {k: v for k, v in mixed.items() if k != "evals"}
    sh = mixed["shape"]
    line["roofline"] = dict(bound="hbm", kernel=f"k_batched<float, {sh['threads']}, "
                                                f"{sh['rows_per_wave']}, {sh['unroll']}> "
                                                f"(whole persistent launch, {sh['blocks']} "
                                                "workgroups)",
                            achieved=round(op_gbps, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                            frac=round(op_gbps / HBM_PEAK_GBPS, 4), traffic=None,
                            algorithmic_bytes_per_launch=op_bytes,
                            note="operator bytes of all Lanczos matvecs and residual-check "
                                 "applies over the launch time (the graph replay)")
    line["matvec_GBps"] = dict(mixed=round(gbps, 1))
    if not args.no_fp64:
        fp64 = run_batched(J, ctx, w, host, False, args.steps, args.warmup)
        line["fp64"] = {k: v for k, v in fp64.items() if k != "evals"}
        line["speedup_mixed_vs_fp64"] = round(fp64["seconds"] / mixed["seconds"], 3)
        line["matvec_GBps"]["fp64"] = round(fp64["matvec_bytes"] / fp64["seconds"] / 1e9, 1)
        line["mixed_vs_fp64_max_rel_eig_diff"] = float(
            np.abs(mixed["evals"] - fp64["evals"]).max() / np.abs(fp64["evals"]).max())
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_batched(w, host, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def main_casea(args, J, ctx, w, host):
    """Table 1 on the GPU: every published (algorithm, nev, mwin, m) row on the
    ten matrices; N_conv and N_MV as [min, avg, max], beside the paper's."""
    import torch
    rows = json.load(open(os.path.join(ROOT, "tests", "golden", "table1_caseA.json")))["rows"]
    ops = []
    for A11, A12, lam in host["mats"]:
        ops.append((J.jl_op_create_dense(ctx, torch.from_numpy(A11).cuda(), torch.from_numpy(A12).cuda()),
                    lam))
    J.jl_solve(ops[0][0], 5, 50, 10, w["tol"], which="largest")   # warm-up
    table, t_jsym, n_jsym = [], 0.0, 0
    t_start = time.perf_counter()
    for alg, nev, mwin, m, *paper in rows:
        standard = alg == "TRLAN"
        conv, mv, incomplete = [], [], 0
        for op, lam in ops:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = J.jl_solve(op, nev, m, mwin, w["tol"], which="largest", standard=standard)
            dt = time.perf_counter() - t0
            if out.status != J.JL_OK:
                raise RuntimeError(f"{alg} {nev}/{mwin}/{m} did not converge: {out.status}")
            top = lam[::-1]
            # every returned value is an eigenvalue of A (true residual below tol)
            if np.abs(out.evals[:, None] - top[None, :]).min(axis=1).max() > 1e-12:
                raise RuntimeError(f"{alg} {nev}/{mwin}/{m}: eigenvalues off the known spectrum")
            if standard:
                # the standard method may stop before the second copy of every
                # pair has entered its Krylov space (a single-vector Krylov
                # space holds one direction per eigenspace until rounding adds
                # the other): count such solves instead of failing them
                if np.abs(np.sort(out.evals)[::-1] - np.repeat(top[:nev // 2], 2)).max() > 1e-12:
                    incomplete += 1
            elif np.abs(out.evals - top[:nev]).max() > 1e-12:
                raise RuntimeError(f"{alg} {nev}/{mwin}/{m}: not the {nev} largest eigenvalues")
            conv.append(out.stats["cycles"])
            mv.append(out.stats["n_mv"])
            if not standard:
                t_jsym += dt
                n_jsym += 1
        row = dict(algorithm=alg, nev=nev, mwin=mwin, m=m,
                   n_conv=[min(conv), round(float(np.mean(conv)), 1), max(conv)],
                   n_mv=[min(mv), round(float(np.mean(mv)), 1), max(mv)],
                   paper_n_conv=paper[0:3], paper_n_mv=paper[3:6])
        if standard:
            row["incomplete_pairs_solves"] = incomplete
        table.append(row)
    total = time.perf_counter() - t_start
    value = t_jsym / n_jsym
    jsym_mv = np.mean([r["n_mv"][1] for r in table if r["algorithm"] == "TRLAN-JSYM" and r["nev"] == 10])
    std_mv = np.mean([r["n_mv"][1] for r in table if r["algorithm"] == "TRLAN" and r["nev"] == 20])
    line = dict(metric=METRIC, value=round(value, 5), unit="s", n_gpus=1, steps=len(rows) * len(ops),
                warmup=1, ms_per_step=round(value * 1e3, 3), higher_is_better=False, scaling="weak",
                vs_baseline=None, dtype="f64", data="synthetic",
                config=dict(workload=describe(w), name=args.workload, n=w["n"], parallelism="1 GPU"),
                note="value: mean time of one TRLAN-JSYM solve over the grid rows and matrices",
                total_seconds=round(total, 2),
                mv_ratio_standard_over_jsym=round(float(std_mv / jsym_mv), 3),
                table1=table)
    print(json.dumps(line), flush=True)


def cpu_baseline_batched(w, host, budget_s):
    """The FP64 oracle (Algorithms 1 and 2, literal MGS) solving the problems
    one after another for about budget_s seconds; the per-problem mean time
    is scaled to the whole batch (labelled extrapolated)."""
    from oracle import jsym, trlan
    t0 = time.perf_counter()
    done = 0
    for A11, A12 in host["probs"][::-1]:   # random order is fine; sizes are i.i.d.
        A = jsym.dense_from_blocks(A11, A12)
        trlan.trlan_jsym(lambda v: A @ v, A.shape[0], w["nev"], w["mwin"], w["m"], w["tol_fp64"],
                         tol_relative=True)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    blas_threads, phys, logical = host_cores()
    return dict(value=dt / done * w["count"], unit="s", cores=blas_threads, kind="oracle",
                sample=f"{done} of {w['count']} problems solved by the FP64 oracle in {dt:.1f} s, "
                       f"mean time per problem scaled to {w['count']} (extrapolated); "
                       f"{blas_threads} BLAS threads on {phys} physical cores / {logical} logical CPUs")


def main_cycles(args, J, ctx, w, host):
    """Stencil workloads: a step is one outer iteration of Algorithm 1.  The
    mixed solve runs to convergence (value = its wall time); the FP64 solve
    runs the same warmup + steps iterations."""
    print(f"[bench] {describe(w)}: mixed solve (to {w['nev']} converged pairs)", file=sys.stderr,
          flush=True)
    mixed = run_cycles(J, ctx, w, host, True, args.steps, args.warmup, args.verbose, full=True)
    st = mixed["stats"]
    print(f"[bench] mixed: {mixed['wall']:.2f} s, {st['cycles']} iterations, {st['n_mv']} matvecs",
          file=sys.stderr, flush=True)
    rates = kernel_rates(st)
    dom = max(("dots", "update"), key=lambda k: st[f"t_{k}"])
    achieved = rates[dom]["gbps"]
    mv_reorth = (st["bytes_matvec"] + st["bytes_dots"] + st["bytes_update"]) / (
        st["t_matvec"] + st["t_dots"] + st["t_update"]) / 1e9
    roof = dict(bound="hbm", kernel=f"reorth_{dom}", achieved=round(achieved, 1),
                peak=HBM_PEAK_GBPS, unit="GB/s", frac=round(achieved / HBM_PEAK_GBPS, 4),
                traffic=traffic_for(dom, args.workload),
                algorithmic_bytes_per_launch=rates[dom]["bytes_per_launch"],
                avg_launch_us=round(rates[dom]["avg_us"], 2), launches=rates[dom]["launches"],
                note="HIP events on the solver's stream around the launches of every "
                     f"{TIMING_STRIDE}th Lanczos step of the mixed solve")
    last = mixed["last"]
    line = dict(
        metric=METRIC, value=round(mixed["wall"], 3), unit="s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(mixed["step"] * 1e3, 2), higher_is_better=False,
        scaling="weak", vs_baseline=None, dtype="fp32+fp64", data="synthetic",
        config=dict(workload=describe(w), name=args.workload, n=mixed["n"], nev=w["nev"], m=w["m"],
                    mwin=w["mwin"], parallelism="1 GPU",
                    step=f"one outer iteration of Alg. 1 (iterations {args.warmup + 1}.."
                         f"{args.warmup + args.steps} of the mixed solve timed; value: the wall "
                         f"time of the whole mixed solve to {w['nev']} converged pairs)"),
        mixed=dict(seconds=mixed["wall"], ms_per_iteration=round(mixed["step"] * 1e3, 2),
                   cycles=st["cycles"], n_mv=st["n_mv"], gs_passes=st["gs_passes"],
                   n_resid=st["n_resid"], res_max=float(last.res.max()), kernels=rates),
        matvec_GBps=dict(mixed=round(rates["matvec"]["gbps"], 1)),
        matvec_plus_reorth_GBps=dict(mixed=round(mv_reorth, 1),
                                     frac=round(mv_reorth / HBM_PEAK_GBPS, 4)),
        roofline=roof,
    )
    del last
    mixed["last"] = None
    if not args.no_fp64:
        print(f"[bench] fp64 solve: the first {args.warmup + args.steps} iterations",
              file=sys.stderr, flush=True)
        fp64 = run_cycles(J, ctx, w, host, False, args.steps, args.warmup, args.verbose,
                          full=False)
        s64 = fp64["stats"]
        r64 = kernel_rates(s64)
        line["fp64"] = dict(ms_per_iteration=round(fp64["step"] * 1e3, 2), cycles=s64["cycles"],
                            n_mv=s64["n_mv"], gs_passes=s64["gs_passes"], kernels=r64,
                            seconds_for_iterations=round(fp64["wall"], 3))
        line["matvec_GBps"]["fp64"] = round(r64["matvec"]["gbps"], 1)
        line["speedup_mixed_vs_fp64"] = round(fp64["step"] / mixed["step"], 3)
        # the same iterations in both precisions: matvecs up to the last timed one
        nc = args.warmup + args.steps
        line["same_iterations_check"] = dict(
            iterations=nc, mixed_seconds=round(float(mixed["cycle_times"][nc - 1]), 3),
            fp64_seconds=round(float(fp64["cycle_times"][nc - 1]), 3))
    if not args.no_cpu:
        print("[bench] cpu oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, host, st, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def kernel_rates(stats):
    out = {}
    for k in ("matvec", "dots", "update"):
        t, nl, b = stats[f"t_{k}"], stats[f"n_{k}_launch"], stats[f"bytes_{k}"]
        if t > 0 and nl > 0:
            out[k] = dict(gbps=b / t / 1e9, avg_us=t / nl * 1e6, bytes_per_launch=b / nl, launches=nl)
    if stats["t_cg"] > 0 and stats["cg_iters"] > 0:
        out["cg"] = dict(gbps=stats["bytes_cg"] / stats["t_cg"] / 1e9,
                         avg_us_per_iter=stats["t_cg"] / stats["cg_iters"] * 1e6,
                         bytes_per_iter=stats["bytes_cg"] / stats["cg_iters"],
                         iters=stats["cg_iters"], max_iters=stats["cg_max_iters"],
                         seconds=stats["t_cg"])
    if stats["t_gemm"] > 0:
        out["gemm"] = dict(tflops=stats["flops_gemm"] / stats["t_gemm"] / 1e12,
                           seconds=stats["t_gemm"], launches=stats["n_gemm_launch"])
    out["ritz_seconds"] = stats["t_ritz"]
    out["resid_seconds"] = stats["t_resid"]
    return out


def traffic_for(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on this workload and on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    src = os.path.join(ROOT, "paper_2001_07428_amd", "csrc", "k_reorth.hip")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if rec.get("source_sha256") != h or rec.get("bench_workload") != workload:
            return None
        return rec.get("hbm_bytes_per_launch")
    except (OSError, ValueError):
        return None


def host_cores():
    """(BLAS threads the oracle's NumPy calls use, physical cores, logical CPUs)."""
    try:
        from threadpoolctl import threadpool_info
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas = None
    try:
        import psutil
        phys = psutil.cpu_count(logical=False)
    except Exception:
        phys = None
    return blas, phys, os.cpu_count()


def cpu_baseline(w, host, gpu_stats, budget_s):
    """The FP64 oracle (literal Algorithm 2) on a bounded prefix of the same
    workload: per-step cost fit a + b*j over the first Lanczos steps, then
    extrapolated to the GPU run's N_MV and sum of basis widths."""
    from oracle import cg, jsym, trlan
    blas_threads, phys, logical = host_cores()
    if w["kind"] == "stencil":
        U, B, L = host["U"], host["B"], w["L"]
        n = 2 * int(np.prod(L)) * 4
        apply = lambda v: jsym.stencil_apply(U, B, L, v)
    elif w["kind"] == "tek":
        from oracle import tek
        Us, kap, na = host["U"], w["kappa"], w["N"] ** 2 - 1
        n = 4 * na
        apply = lambda v: tek.to_canonical(
            tek.apply_A(Us, kap, tek.from_canonical(v, na), entries=True), na)
    else:
        A = jsym.dense_from_blocks(host["A11"], host["A12"])
        n = A.shape[0]
        apply = lambda v: A @ v
    step = apply
    if w.get("invert"):   # invert mode: every Lanczos step solves by the oracle's CG
        step = lambda v: cg.cg(apply, v, w.get("cg_tol_fp64", w["cg_tol"]), 100000)[0]
    smax = 64
    V = np.zeros((n, smax + 1), dtype=np.complex128)
    T = np.zeros((smax + 1, smax))
    V[:, 0] = 1.0 / np.sqrt(n)
    stats = dict(n_mv=0, gs_passes=0)
    times = []
    t_start = time.perf_counter()
    j = 0
    while j < smax and time.perf_counter() - t_start < budget_s:
        t0 = time.perf_counter()
        trlan.lanczos_jsym(step, V, T, j, j + 1, stats)
        times.append((j, time.perf_counter() - t0))
        j += 1
    js = np.array([t[0] for t in times], float)
    ts = np.array([t[1] for t in times], float)
    if len(js) >= 2:
        b, a = np.polyfit(js, ts, 1)
        b = max(b, 0.0)
    else:
        a, b = float(ts.mean()), 0.0
    nmv = gpu_stats["n_mv"]
    sum_j = gpu_stats["sum_ncol"] - nmv
    est = a * nmv + b * sum_j
    return dict(value=est, unit="s", cores=blas_threads, kind="oracle",
                sample=(f"first {len(js)} Lanczos steps (Alg. 2, literal MGS, FP64"
                        f"{', each with a CG solve' if w.get('invert') else ''}) of the same "
                        f"workload in {time.perf_counter() - t_start:.1f} s; per-step time fit "
                        f"{a:.3g} + {b:.3g}*j s extrapolated to the GPU run's N_MV={nmv} and "
                        f"sum j={sum_j} (extrapolated); {blas_threads} BLAS threads on "
                        f"{phys} physical cores / {logical} logical CPUs"))


def probe(w, reps=3):
    """Kernel probe for hardware counters: a plain 1 GiB elementwise pass,
    y = -x (HBM calibration: 1 GiB read, 1 GiB written), then `reps` operator applies and J-restricted Gram-Schmidt
    passes at the workload's shape (mixed precision, basis width 3m/4), and
    `reps` restart products V_m Z (m basis vectors, k = 3m/5 Ritz vectors)."""
    import torch
    from paper_2001_07428_amd import jlanczos as J
    host = make_host_inputs(w)
    ctx = J.Context(0)
    x = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").uniform_()
    y = torch.empty_like(x)
    for _ in range(reps):   # y = -x: one elementwise kernel reading and writing 1 GiB
        torch.neg(x, out=y)
    del x, y
    op = make_op(J, ctx, w, host, torch.complex64)
    ncol = (3 * w["m"]) // 4
    kz = (3 * w["m"]) // 5
    g = torch.Generator(device="cuda:0").manual_seed(0)
    V = torch.randn((w["m"], op.n), dtype=torch.complex64, device="cuda:0", generator=g) / np.sqrt(op.n)
    u = torch.randn(op.n, dtype=torch.complex64, device="cuda:0", generator=g)
    for _ in range(reps):
        J.jl_op_apply(op, V[0], u)
        J.jl_reorth_pass(ctx, V[:ncol], u)
    Z = torch.randn((w["m"], kz), dtype=torch.float64, device="cuda:0", generator=g)
    for _ in range(reps):
        Y = J.jl_basis_update(ctx, V, Z)
        del Y
    torch.cuda.synchronize()
    print(json.dumps(dict(probe=w, ncol=ncol, gemm_m=w["m"], gemm_k=kz, n=op.n, reps=reps,
                          copy_bytes=2 * (1 << 30))), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 10 outer iterations for the stencils, else 2)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="warm-up steps (default: 2 outer iterations for the stencils, else 1)")
    ap.add_argument("--workload", default="stencil32", choices=sorted(WORKLOADS))
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison solve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--verbose", action="store_true",
                    help="per-iteration progress on stderr (always on for the stencil workloads, "
                         "whose solves take minutes, unless --quiet)")
    ap.add_argument("--quiet", action="store_true", help="no per-iteration progress")
    ap.add_argument("--probe", action="store_true",
                    help="run the counter probe (copy + apply + reorth pass) instead")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); the multi-GPU "
              "sharding of this solver is a design, not a build.", file=sys.stderr)
        sys.exit(2)
    w = WORKLOADS[args.workload]
    cyc = w.get("step") == "cycle"
    if args.steps is None:
        args.steps = 10 if cyc else 2
    if args.warmup is None:
        args.warmup = 2 if cyc else 1
    if cyc and not args.quiet:
        args.verbose = True
    if args.steps < (1 if cyc else 0) or args.warmup < 0:
        ap.error("--steps must be >= 1 for the stencil workloads (>= 0 otherwise), --warmup >= 0")
    # host inputs first: the Case A recipe runs in worker processes, forked
    # before anything in this process touches the GPU
    host = None if args.probe else make_host_inputs(w)
    import torch
    from paper_2001_07428_amd import jlanczos as J
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    J.load_library()
    if args.probe:
        probe(w)
        return
    ctx = J.Context(0)
    if w["kind"] == "batched":
        main_batched(args, J, ctx, w, host)
        return
    if w["kind"] == "casea":
        main_casea(args, J, ctx, w, host)
        return
    if w.get("step") == "cycle":
        main_cycles(args, J, ctx, w, host)
        return
    print(f"[bench] {describe(w)}: mixed solves", file=sys.stderr, flush=True)
    mixed = run_precision(J, ctx, w, host, True, args.steps, args.warmup, args.verbose)
    fp64 = None
    if not args.no_fp64:
        print("[bench] fp64 solves", file=sys.stderr, flush=True)
        fp64 = run_precision(J, ctx, w, host, False, args.steps, args.warmup, args.verbose)
    rates = kernel_rates(mixed["stats"])
    if w["kind"] == "tek":   # bound by the matrix products of the operator apply
        st = mixed["stats"]
        N = w["N"]
        flops = 512.0 * N ** 3       # 64 complex N x N products per apply of A (half-spinors)
        if w.get("invert"):
            per, what = st["t_cg"] / st["cg_iters"], "CG iteration (apply + fused update)"
        else:
            per, what = st["t_matvec"] / st["n_matvec_launch"], "operator apply"
        achieved = flops / per / 1e12
        roof = dict(bound="mfma", kernel=f"k_zgemm (TEK {what}, FP32 MFMA)",
                    achieved=round(achieved, 2), peak=157.3, unit="TFLOP/s",
                    frac=round(achieved / 157.3, 4), traffic=None,
                    algorithmic_flops_per_launch=flops, avg_launch_us=round(per * 1e6, 1),
                    note="flops of the unpadded products over the whole apply (conversions "
                         "and combines included)")
    elif "cg" in rates:   # invert mode: the CG loop dominates
        achieved = rates["cg"]["gbps"]
        roof = dict(bound="hbm", kernel="cg_iteration (apply + alpha/update/beta/direction)",
                    achieved=round(achieved, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBPS, 4), traffic=None,
                    algorithmic_bytes_per_launch=rates["cg"]["bytes_per_iter"],
                    avg_launch_us=round(rates["cg"]["avg_us_per_iter"], 2),
                    note="per CG iteration (three launches), launch gaps included")
    else:
        dom = max(("dots", "update"), key=lambda k: mixed["stats"][f"t_{k}"])
        achieved = rates[dom]["gbps"]
        roof = dict(bound="hbm", kernel=f"reorth_{dom}", achieved=round(achieved, 1),
                    peak=HBM_PEAK_GBPS, unit="GB/s", frac=round(achieved / HBM_PEAK_GBPS, 4),
                    traffic=traffic_for(dom, args.workload),
                    algorithmic_bytes_per_launch=rates[dom]["bytes_per_launch"],
                    avg_launch_us=round(rates[dom]["avg_us"], 2))
    line = dict(
        metric=METRIC, value=round(mixed["seconds"], 4), unit="s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(mixed["seconds"] * 1e3, 2), higher_is_better=False,
        scaling="weak", vs_baseline=None, dtype="fp32+fp64", data="synthetic",
        config=dict(workload=describe(w), name=args.workload, n=mixed["n"], nev=w["nev"], m=w["m"],
                    mwin=w["mwin"], parallelism="1 GPU"),
        mixed=dict(seconds=mixed["seconds"], cycles=mixed["last"].stats["cycles"],
                   cg_iters=mixed["last"].stats["cg_iters"],
                   n_mv=mixed["last"].stats["n_mv"], gs_passes=mixed["last"].stats["gs_passes"],
                   res_max=float(mixed["last"].res.max()), kernels=rates),
        matvec_GBps=dict(mixed=round(rates["matvec"]["gbps"], 1)) if "matvec" in rates else {},
        roofline=roof,
    )
    if fp64 is not None:
        r64 = kernel_rates(fp64["stats"])
        line["fp64"] = dict(seconds=fp64["seconds"], cycles=fp64["last"].stats["cycles"],
                            cg_iters=fp64["last"].stats["cg_iters"],
                            n_mv=fp64["last"].stats["n_mv"], gs_passes=fp64["last"].stats["gs_passes"],
                            res_max=float(fp64["last"].res.max()), kernels=r64)
        if "matvec" in r64:
            line["matvec_GBps"]["fp64"] = round(r64["matvec"]["gbps"], 1)
        line["speedup_mixed_vs_fp64"] = round(fp64["seconds"] / mixed["seconds"], 3)
        e32, e64 = mixed["last"].evals, fp64["last"].evals
        line["mixed_vs_fp64_max_rel_eig_diff"] = float(np.abs(e32 - e64).max() / np.abs(e64).max())
    if not args.no_cpu:
        print("[bench] cpu oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, host, mixed["last"].stats, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
