"""Autotuner for the batched solver's launch shape and apply tile.

Knobs (jl_batch_shape):
  threads           workgroup size, 128 / 256 / 512: more wavefronts per problem
                    shorten each matvec and Gram-Schmidt pass but leave fewer
                    workgroups per compute unit;
  blocks            persistent workgroups, 1, 2 or 3 per compute unit (capped by
                    the problem count);
  rows_per_wave     rows of [A11 A12] a wavefront applies at once (1 or 2: two rows
                    share the operand reads and double the loads in flight);
  unroll            column steps whose matrix loads a lane issues together (4 or 8);
  lds_matrix_bytes  LDS per workgroup for a problem's whole [A11 A12]: problems whose
                    matrices fit are read from LDS for their whole solve (0, 32 KiB,
                    64 KiB), at the price of LDS per workgroup.

The search is staged (each stage keeps the best of the previous one): launch shape
(threads x workgroups per CU), then the apply tile (rows per wave x unroll), then the
LDS residency threshold.  Every candidate is timed on the caller's batch (replays of
the captured graph, median of `reps`) and the fastest is recorded in a JSON cache keyed
by the device and a signature of the batch: count, the histogram of log2 of the problem
sizes (the size buckets), nev, m and dtype.

    python -m paper_2001_07428_amd.tune   # on a GPU; the defaults are the 512-problem benchmark batch

Batch(..., shape=None) looks the shape up in the cache (tuned.json next to this file)
and falls back to the library defaults, with a warning, when the signature is absent.
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
TILES = ((1, 4), (1, 8), (2, 4), (2, 8))          # (rows_per_wave, unroll)
LDS_MATRIX = (0, 32 * 1024, 64 * 1024)


def signature(n, nev, m, dtype_name):
    """Batch signature: count, log2-size histogram (size buckets), nev, m, dtype."""
    n = np.asarray(n)
    hist = np.bincount(np.floor(np.log2(n)).astype(int), minlength=12)[:12].tolist()
    return f"count={len(n)};hist={hist};nev={nev};m={m};dtype={dtype_name}"


def device_key():
    """Architecture and compute-unit count (the marketing name is left out: it
    depends on the driver's device-id table, which some systems lack)."""
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "") or ""
    return f"{arch.split(':')[0]}|cu={p.multi_processor_count}"


def lookup(n, nev, m, dtype_name):
    """The cached jl_batch_shape (a dict) for this batch and device, or None."""
    try:
        cache = json.load(open(CACHE))
    except (OSError, ValueError):
        return None
    rec = cache.get(device_key(), {}).get(signature(n, nev, m, dtype_name))
    return dict(rec["shape"]) if rec and "shape" in rec else None


def _time(J, ctx, A11s, A12s, nev, m, mwin, tol, tol_relative, shape, reps):
    import torch
    try:
        b = J.Batch(ctx, A11s, A12s, nev, m, mwin, tol, tol_relative=tol_relative, shape=shape)
    except J.JLError:   # e.g. more LDS than a workgroup may use
        return None
    b.run()   # warm-up
    times = []
    rc = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, *_ = b.run()
        times.append(time.perf_counter() - t0)
    b.close()
    return dict(shape=dict(shape), seconds=statistics.median(times), status=rc)


def tune(ctx, A11s, A12s, nev, m, mwin, tol, tol_relative=False, reps=3, verbose=True):
    import torch
    from . import jlanczos as J
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    count = len(A11s)
    results = []

    def run(shape):
        r = _time(J, ctx, A11s, A12s, nev, m, mwin, tol, tol_relative, shape, reps)
        if r is None:
            return None
        results.append(r)
        if verbose:
            print(f"[tune] {shape}: {r['seconds'] * 1e3:8.2f} ms", flush=True)
        return r

    def best():
        ok = [r for r in results if r["status"] == J.JL_OK] or results
        return min(ok, key=lambda r: r["seconds"])

    seen = set()
    for threads in THREADS:                       # stage 1: launch shape
        for per in PER_CU:
            shape = dict(threads=threads, blocks=min(count, per * ncu), rows_per_wave=1, unroll=4,
                         lds_matrix_bytes=0)
            key = tuple(sorted(shape.items()))
            if key not in seen:
                seen.add(key)
                run(shape)
    base = best()["shape"]
    for rpw, unr in TILES:                        # stage 2: apply tile
        shape = dict(base, rows_per_wave=rpw, unroll=unr)
        key = tuple(sorted(shape.items()))
        if key not in seen:
            seen.add(key)
            run(shape)
    base = best()["shape"]
    for lds in LDS_MATRIX:                        # stage 3: LDS-resident matrices
        shape = dict(base, lds_matrix_bytes=lds)
        key = tuple(sorted(shape.items()))
        if key not in seen:
            seen.add(key)
            run(shape)
    return best(), results


def save(n, nev, m, dtype_name, best, results):
    try:
        cache = json.load(open(CACHE))
    except (OSError, ValueError):
        cache = {}
    cache.setdefault(device_key(), {})[signature(n, nev, m, dtype_name)] = dict(
        shape=best["shape"], seconds=best["seconds"],
        candidates=[dict(shape=r["shape"], seconds=r["seconds"]) for r in results])
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
