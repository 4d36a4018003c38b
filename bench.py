#!/usr/bin/env python3
"""Benchmark of the plain two-phase SpGEMM C = A*A on one MI355X.

Default workload: A = 2D 5-point Laplacian on a 1024 x 1024 grid (1,048,576
rows, 5,238,784 nonzeros, FP64), C = A*A (26,177,544 intermediate products,
13,611,012 nonzeros).  Inputs are generated on the host, copied to HBM once,
and every timed step is one full msp_spgemm call (statistics, binning,
symbolic pass, prefix sum, allocation of C, numeric pass with sorted rows).

Prints ONE JSON line with the whole-job throughput (GFLOP/s = 2 x products /
time), the HBM roofline of the dominant kernel (the numeric pass, timed with
HIP events on the library's stream), and the CPU oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, vendor figure

# FETCH_SIZE / WRITE_SIZE of the numeric kernel on the default workload,
# from two rocprofv3 --pmc passes scaled by a plain copy kernel (see
# profiles/); None until measured for the current kernel.
MEASURED_TRAFFIC_BYTES = None


def workload(name: str):
    from paper_2112_10037_amd import gen
    if name == "laplacian2d_1024":
        return ("2D 5-point Laplacian 1024x1024, C = A*A, FP64",
                gen.laplacian_2d(1024))
    if name == "er4096":
        return ("Erdos-Renyi 4096x4096, 8 nnz/row, FP64 U[-1,1], seed 0, C = A*A",
                gen.erdos_renyi(4096, 4096, 8, seed=0))
    if name == "rmat20":
        return ("R-MAT 2^20, 16*2^20 edges, (0.57,0.19,0.19,0.05), FP32 (0,1], seed 1, C = A*A",
                gen.rmat(20, 16 << 20, seed=1))
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(A, nnz_c: int) -> int:
    """|A| + |B| + |C| with B = A counted again: row pointers (int64),
    column indices (int32) and values of each operand."""
    vb = A.val.dtype.itemsize
    a = (A.nrows + 1) * 8 + A.nnz * (4 + vb)
    c = (A.nrows + 1) * 8 + nnz_c * (4 + vb)
    return 2 * a + c


def cpu_baseline(A, products: int, budget_s: float) -> dict:
    import oracle
    cores = oracle.num_threads()
    t0 = time.perf_counter()
    runs = 0
    while True:
        oracle.spgemm(A, A)
        runs += 1
        el = time.perf_counter() - t0
        if el >= budget_s or runs >= 200:
            break
    return {"value": round(2.0 * products * runs / el / 1e9, 3), "unit": "GFLOP/s",
            "cores": cores, "kind": "oracle",
            "sample": f"{runs} full products of the same workload in {el:.1f} s "
                      f"(C oracle, FP64 dense accumulator, OpenMP over rows)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="laplacian2d_1024")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tuning", default=None,
                    help="hash_scale,group_scale,spill_nnz,block_rows,merge_k (default: library's)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the product would shard).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2112_10037_amd import binding
    import oracle

    desc, A = workload(args.workload)
    st = oracle.row_stats(A, A)
    products = int(st["prod"].sum())
    dA = binding.DeviceCSR.from_host(A, "cuda:0")
    h = binding.Handle(0)
    if args.tuning:
        h.set_tuning(tuple(int(x) for x in args.tuning.split(",")))

    for _ in range(args.warmup):
        C = h.spgemm(dA, dA)
    h.sync()
    nnz_c = C.nnz
    del C

    h.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        C = h.spgemm(dA, dA, check=False)
        del C
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    h.sync()          # raises if any timed call flagged an internal error
    prof = h.profile_get()
    h.profile(False)

    ms_step = el * 1e3 / args.steps
    gflops = 2.0 * products / (el / args.steps) / 1e9
    num_ms, num_n = prof["numeric"]
    num_avg_s = num_ms / max(num_n, 1) / 1e3
    alg = algorithmic_bytes(A, nnz_c)
    achieved = alg / num_avg_s / 1e9
    traffic = MEASURED_TRAFFIC_BYTES if args.workload == "laplacian2d_1024" else None

    out = {
        "metric": "SpGEMM GFLOP/s (2x products/s)",
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if A.val.dtype == np.float64 else "f32",
        "data": "synthetic",
        "config": {"workload": desc, "rows": A.nrows, "nnz_a": A.nnz, "products": products,
                   "nnz_c": nnz_c, "path": "plain two-phase",
                   "tuning": list(h.get_tuning())},
        "roofline": {"bound": "hbm", "kernel": "numeric pass",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes": alg,
                     "avg_launch_ms": round(num_avg_s * 1e3, 5)},
        "phases_ms_per_step": {k: round(v[0] / args.steps, 5) for k, v in prof.items() if v[1]},
        "hbm_gbs_whole_step_algorithmic": round(alg / (el / args.steps) / 1e9, 1),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(A, products, args.cpu_seconds)
    if args.calibrate_copy:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = src.numel() * 8
    h.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
