"""Batched products: packed Galerkin batches and the autotuner's JSON cache
(argument marshalling and orchestration; the products run in the library).
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import binding, gen

# Candidate tunings searched by default: the merge accumulator (K = 8, 4, or
# off) crossed with the hash-table and lane-group scales.
CANDIDATES = [(hs, gs, 4096, 128, mk) for mk in (8, 4, -1) for hs in (1, 2) for gs in (0, 1)]


def galerkin_host(sides, dtype=np.float64):
    """Host (A, P, R) lists for sides n (one 7-point Laplacian problem per
    side; problems with equal sides share their host arrays)."""
    cache = {}
    A, P, R = [], [], []
    for n in sides:
        n = int(n)
        if n not in cache:
            cache[n] = gen.galerkin_problem(n, dtype)
        a, p, r = cache[n]
        A.append(a)
        P.append(p)
        R.append(r)
    return A, P, R


def galerkin_batch(sides, dtype=np.float64, device="cuda"):
    """Packed device batches (A, P, R) of the Galerkin products R (A P)."""
    A, P, R = galerkin_host(sides, dtype)
    return tuple(binding.PackedBatch.from_host(x, device) for x in (A, P, R))


def signature(*batches) -> str:
    """Shape key of a batch: problem rows, columns and nonzeros."""
    h = hashlib.sha256()
    for b in batches:
        if b is None:
            h.update(b"none")
            continue
        h.update(np.ascontiguousarray(b.row_start).tobytes())
        h.update(np.ascontiguousarray(b.ncols).tobytes())
        h.update(str(b.nnz).encode())
    return h.hexdigest()[:24]


def autotune_cached(h: binding.Handle, A, P, R, path: str, candidates=CANDIDATES, reps=5):
    """Best tuning for the batch's shape: from the JSON cache at `path` when
    it holds one for this signature, else measured and stored.
    Returns (tuning, info) where info says whether it was cached."""
    key = signature(A, P, R)
    cache = {}
    if path and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        return binding.tuning_from_json(json.dumps(cache[key]["tuning"])), {"cached": True}
    best, times = binding.autotune(h, A, P, R, candidates, reps=reps)
    cache[key] = {"tuning": json.loads(binding.tuning_to_json(best)),
                  "candidates": [list(c) for c in candidates], "median_ms": times}
    if path:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, {"cached": False, "median_ms": times}


def main(argv=None):
    """Build the Galerkin batch R (A P) of `--problems` problems (sides
    ~ U{16..64}, seed 5), plan it once and time `--replays` graph replays."""
    import argparse
    import time
    import torch
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--problems", type=int, default=512)
    ap.add_argument("--replays", type=int, default=6)
    ap.add_argument("--tuning", default="1,0,4096,128,8",
                    help="hash_scale,group_scale,spill_nnz,block_rows,merge_k")
    a = ap.parse_args(argv)
    tuning = tuple(int(x) for x in a.tuning.split(","))
    sides = gen.galerkin_sizes(a.problems, 16, 64, seed=5)
    h = binding.Handle(0)
    pA, pP, pR = galerkin_batch(sides)
    plan = binding.Batch(h, pA, pP, pR, tuning=tuning)
    print("plan", plan.info(), flush=True)
    for i in range(a.replays):
        t0 = time.perf_counter()
        plan.execute()
        plan.sync()
        torch.cuda.synchronize()
        print(f"replay {i}: {(time.perf_counter() - t0) * 1e3:.3f} ms", flush=True)
    plan.close()
    h.close()


if __name__ == "__main__":
    main()
