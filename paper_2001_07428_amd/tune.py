"""Autotuner for the batched solver's launch shape.

The batched kernel has two knobs: the workgroup size (128, 256 or 512
threads: more wavefronts per problem shorten each matvec and Gram-Schmidt pass
but leave fewer workgroups per CU) and the number of persistent workgroups
(the grid: 1, 2 or 3 per compute unit, capped by the problem count).  The tuner
times every combination on the caller's batch (replays of the captured graph,
median of `reps`) and records the fastest in a JSON cache keyed by the device
name and a signature of the batch (count, size histogram, nev, m, dtype).

    python -m paper_2001_07428_amd.tune   # on a GPU; the defaults are the 512-problem benchmark batch

Batch(..., threads=0, blocks=0) looks the shape up in the cache (tuned.json
next to this file) and falls back to the library default (256 threads,
2 workgroups per CU) when the signature is absent.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")
THREADS = (128, 256, 512)
PER_CU = (1, 2, 3)


def signature(n, nev, m, dtype_name):
    """Batch signature: count, log2-size histogram, nev, m, dtype."""
    n = np.asarray(n)
    hist = np.bincount(np.floor(np.log2(n)).astype(int), minlength=12)[:12].tolist()
    return f"count={len(n)};hist={hist};nev={nev};m={m};dtype={dtype_name}"


def device_key():
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "") or ""
    return f"{p.name}|{arch.split(':')[0]}|cu={p.multi_processor_count}"


def lookup(n, nev, m, dtype_name):
    """(threads, blocks) from the cache, or None."""
    try:
        cache = json.load(open(CACHE))
    except (OSError, ValueError):
        return None
    rec = cache.get(device_key(), {}).get(signature(n, nev, m, dtype_name))
    return (rec["threads"], rec["blocks"]) if rec else None


def tune(ctx, A11s, A12s, nev, m, mwin, tol, tol_relative=False, reps=3, verbose=True):
    import torch
    from . import jlanczos as J
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    count = len(A11s)
    results = []
    for threads in THREADS:
        for per in PER_CU:
            blocks = min(count, per * ncu)
            if results and any(r["threads"] == threads and r["blocks"] == blocks for r in results):
                continue
            b = J.Batch(ctx, A11s, A12s, nev, m, mwin, tol, tol_relative=tol_relative,
                        threads=threads, blocks=blocks)
            b.run()   # warm-up
            times = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc, *_ = b.run()
                times.append(time.perf_counter() - t0)
            b.close()
            rec = dict(threads=threads, blocks=blocks, seconds=statistics.median(times), status=rc)
            results.append(rec)
            if verbose:
                print(f"[tune] threads {threads:4d} blocks {blocks:5d}: {rec['seconds'] * 1e3:8.2f} ms",
                      flush=True)
    ok = [r for r in results if r["status"] == J.JL_OK] or results
    return min(ok, key=lambda r: r["seconds"]), results


def save(n, nev, m, dtype_name, best, results):
    try:
        cache = json.load(open(CACHE))
    except (OSError, ValueError):
        cache = {}
    cache.setdefault(device_key(), {})[signature(n, nev, m, dtype_name)] = dict(
        threads=best["threads"], blocks=best["blocks"], seconds=best["seconds"],
        candidates=[{k: r[k] for k in ("threads", "blocks", "seconds")} for r in results])
    with open(CACHE, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def main():
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch
    from paper_2001_07428_amd import inputs, jlanczos as J
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--nev", type=int, default=8)
    ap.add_argument("--m", type=int, default=32)
    ap.add_argument("--mwin", type=int, default=16)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--precisions", default="c64,c128")
    args = ap.parse_args()
    n, probs = inputs.batched_dense(args.seed, count=args.count)
    ctx = J.Context(0)
    for name in args.precisions.split(","):
        dt = torch.complex64 if name == "c64" else torch.complex128
        tol = args.tol if name == "c64" else 1e-10
        A11s = [torch.from_numpy(a).to("cuda:0", dt) for a, _ in probs]
        A12s = [torch.from_numpy(c).to("cuda:0", dt) for _, c in probs]
        best, results = tune(ctx, A11s, A12s, args.nev, args.m, args.mwin, tol, tol_relative=True,
                             reps=args.reps)
        save(n, args.nev, args.m, name, best, results)
        print(json.dumps(dict(dtype=name, best=best)), flush=True)


if __name__ == "__main__":
    main()
