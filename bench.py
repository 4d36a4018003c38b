#!/usr/bin/env python3
"""Benchmark of the SpGEMM library on one MI355X.

Main line (the `value`): the plain two-phase product C = A*A with A the
R-MAT power-law graph of 2^20 vertices and 16 x 2^20 drawn edges,
(a, b, c, d) = (0.57, 0.19, 0.19, 0.05), duplicates merged, FP32 values in
(0, 1], seed 1: 1,048,576 rows, 16,086,247 nonzeros, 2.09e10 intermediate
products, nnz(C) = 9.7e9 (about 78 GB of C).  Inputs are copied to HBM once;
every timed step is one whole msp_spgemm call (statistics, binning,
symbolic pass, prefix sum, allocation of C, numeric pass with sorted rows),
waited for.  GFLOP/s = 2 x products / median step time.

Also reported on the same line:
  * roofline: the global bin's numeric kernel (k_num_win, the dominant
    kernel), its algorithmic bytes over its average launch time (HIP events
    on the library's stream), against 8 TB/s;
  * cpu_baseline: the C oracle on the host cores, on row blocks of the same
    product streamed one after another (C is never held whole);
  * configs: the Erdos-Renyi 4096 and 2D Laplacian 1024^2 products, each
    timed the same way;
  * learned_vs_plain: the one-pass learned product against the plain one on
    the 16 held-out members of a 64-matrix mixed suite (27-point stencils,
    Erdos-Renyi with 4..32 nonzeros per row, R-MAT with degree 8..32; FP64),
    the network trained on the GPU on the other 48;
  * batched_vs_plain: 512 Galerkin products R (A P) (7-point Laplacians with
    sides n ~ U{16..64}, 2x2x2 aggregation) in one graph replay against the
    1,024 plain calls they amount to.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, vendor figure

# HBM bytes per launch of the dominant kernel of a workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors
# read off a 1 GiB copy kernel), valid only for the kernel sources and the
# tuning whose hash is given; any other state reports null.
# HBM bytes per launch of the roofline kernel, from two rocprofv3 --pmc runs
# (2 x FETCH_SIZE + WRITE_SIZE, the factors a 1 GiB device copy gives in the
# same runs): profiles/rmat20_kernels.md.  Keyed by workload and tuning; a
# figure is reported only while the kernel sources' code is the one measured.
MEASURED_TRAFFIC = {
    ("rmat20", (1, 0, 4096, 1024, 8)): {"bytes": 346818514003, "sources_sha256": "82b603c4619e6c4fe1412518d263c78eb002893834357db25f067a6c05068124"},
    ("rmat20", (1, 0, 2048, 1024, 8)): {"bytes": 350098073402, "sources_sha256": "1263d4858f1712fb7087ae5c807c546148ab4ccaa21c36e4e030f20db324f3f7"},
    ("rmat20", (1, 0, 1024, 1024, 8)): {"bytes": 350993861306, "sources_sha256": "a58847084f2b78983284bafdec280f84aaae1b56ae666730da3cc90a43e7295a"},
}
KERNEL_SOURCES = ["kernels.hpp", "types.hpp", "spgemm.hip", "msp_api.hip", "internal.hpp"]


def _code_only(text: str) -> str:
    """The source without comments, trailing spaces and blank lines (string
    literals in these files hold no comment markers)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_sources_hash(tuning) -> str:
    """Hash of the kernel sources' code and the tuning in effect: a comment
    edit keeps a measured traffic figure valid, any code or tuning change
    does not."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2112_10037_amd", "csrc", name), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    h.update(repr(tuple(int(x) for x in tuning)).encode())
    return h.hexdigest()


def workload(name: str):
    from paper_2112_10037_amd import gen
    if name == "laplacian2d_1024":
        return ("2D 5-point Laplacian 1024x1024, C = A*A, FP64", gen.laplacian_2d(1024))
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


def csr_bytes(nrows: int, nnz: int, vb: int = 8) -> int:
    return (nrows + 1) * 8 + nnz * (4 + vb)


def row_products(A, B) -> np.ndarray:
    """Intermediate products of every row of A*B (host arithmetic on the
    generator's arrays: sum of the B-row lengths each row selects)."""
    blen = np.diff(B.row_ptr).astype(np.int64)
    cs = np.zeros(A.nnz + 1, dtype=np.int64)
    np.cumsum(blen[A.col], out=cs[1:])
    return cs[A.row_ptr[1:]] - cs[A.row_ptr[:-1]]


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, prods: np.ndarray, budget_s: float, block: int = 1024) -> dict:
    """The oracle on the host cores, on a bounded sample: row blocks of
    `block` rows spread evenly over the matrix (a stride through the block
    list, so heavy and light rows are both sampled), each computed and
    dropped before the next, until the time budget is spent.  GFLOP/s = 2 x
    products of the blocks done / their time."""
    import oracle
    cores = oracle.num_threads()
    nblk = (A.nrows + block - 1) // block
    order = np.arange(nblk)
    stride = 97 if nblk % 97 else 89                  # coprime with the block count: every block once
    order = (order * stride) % nblk
    done_p = 0
    done_rows = 0
    blocks = 0
    t_all = 0.0
    for b in order:
        r0, r1 = int(b) * block, min(A.nrows, (int(b) + 1) * block)
        t0 = time.perf_counter()
        ref = oracle.spgemm(A, A, r0, r1)
        t_all += time.perf_counter() - t0
        del ref
        done_p += int(prods[r0:r1].sum())
        done_rows += r1 - r0
        blocks += 1
        if t_all >= budget_s:
            break
    return {"value": round(2.0 * done_p / t_all / 1e9, 3), "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"{blocks} row blocks of {block} rows ({done_rows} rows, {done_p} products, "
                      f"{done_p / max(int(prods.sum()), 1) * 100:.2f}% of the product's) spread evenly over "
                      f"the matrix, streamed one at a time, in {t_all:.1f} s (C oracle: FP64 dense "
                      f"accumulator, OpenMP over rows)",
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def vendor_spgemm(dA, products: int, nnz_c: int, reps: int = 20):
    """The same product through torch.sparse.mm on CSR tensors (hipSPARSE's
    SpGEMM on ROCm), timed over reps calls: context beside the library."""
    import torch
    try:
        T = torch.sparse_csr_tensor(dA.row_ptr, dA.col.to(torch.int64), dA.val, size=(dA.nrows, dA.ncols))
        C = torch.sparse.mm(T, T)
        torch.cuda.synchronize()
        if int(C.values().numel()) != nnz_c:
            return {"error": "nnz differs"}
        for _ in range(2):
            C = torch.sparse.mm(T, T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            C = torch.sparse.mm(T, T)
        torch.cuda.synchronize()
        s = (time.perf_counter() - t0) / reps
        del C, T
        return {"path": "torch.sparse.mm on CSR tensors (hipSPARSE SpGEMM)", "ms": round(s * 1e3, 4),
                "gflops": round(2.0 * products / s / 1e9, 3)}
    except Exception as e:          # a torch build without sparse CSR matmul on the GPU
        return {"error": repr(e)[:200]}


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """GB/s of a plain device-to-device copy (bytes read + written), timed
    with HIP events: the achievable HBM rate the roofline is also read against."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2.0 * nbytes / s / 1e9


# ---------------------------------------------------------------------------
# energy (the paper's Sec. V-C energy per SpGEMM and its utilization factor)
# ---------------------------------------------------------------------------
PEAK_VECTOR_GFLOPS = {"f32": 157300.0, "f64": 78600.0}     # MI355X vendor figures


class EnergyMeter:
    """Board energy of GPU 0 from the SMI energy counter (the accumulator
    times its resolution, in microjoules)."""

    def __init__(self):
        import amdsmi
        self._smi = amdsmi
        amdsmi.amdsmi_init()
        self._h = amdsmi.amdsmi_get_processor_handles()[0]

    def joules(self) -> float:
        e = self._smi.amdsmi_get_energy_count(self._h)
        return e["energy_accumulator"] * e["counter_resolution"] * 1e-6

    def close(self):
        try:
            self._smi.amdsmi_shut_down()
        except Exception:
            pass


def energy_of(meter, fn, min_seconds: float = 3.0, idle_seconds: float = 1.0) -> dict:
    """Energy per call of fn (which waits for its own result), from the
    counter read before and after as many calls as fill min_seconds; the
    idle draw over idle_seconds is measured first, and the energy above it
    is reported as well."""
    import torch
    torch.cuda.synchronize()
    e0, t0 = meter.joules(), time.perf_counter()
    time.sleep(idle_seconds)
    e1, t1 = meter.joules(), time.perf_counter()
    idle_w = (e1 - e0) / (t1 - t0)
    fn()
    n = 0
    e0, t0 = meter.joules(), time.perf_counter()
    while True:
        fn()
        n += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    torch.cuda.synchronize()
    e1, t1 = meter.joules(), time.perf_counter()
    per = (e1 - e0) / n
    per_s = (t1 - t0) / n
    return {"joules_per_call": round(per, 6), "calls": n, "avg_power_w": round((e1 - e0) / (t1 - t0), 1),
            "idle_power_w": round(idle_w, 1), "joules_per_call_above_idle": round(per - idle_w * per_s, 6),
            "seconds_per_call": round(per_s, 6)}


def energy_entry(meter, fn, products: int, dtype: str) -> dict:
    e = energy_of(meter, fn)
    gflops = 2.0 * products / e["seconds_per_call"] / 1e9
    e["gflops_per_watt"] = round(gflops / e["avg_power_w"], 3) if e["avg_power_w"] > 0 else None
    # the paper's utilization factor: operations over (clock x units x time),
    # i.e. the achieved rate over the peak vector rate of the value type
    e["stuf"] = round(gflops / PEAK_VECTOR_GFLOPS[dtype], 6)
    return e


# ---------------------------------------------------------------------------
# the paper's eight matrices, as FP32 stand-ins of the same shapes
# ---------------------------------------------------------------------------
# FSpGEMM on the Arria 10 GX, ms per SpGEMM (Sec. V-C, Table VII): context
# only (the paper's matrices, FLOP convention and product are not ours)
PAPER_FPGA_MS = {"poisson3Da": 5, "2cubes_sphere": 9, "filter3D": 42, "cage12": 15, "scircuit": 6,
                 "mac_econ_fwd500": 7, "offshore": 23, "webbase-1M": 25}


def table4_leg(h, steps: int = 10) -> dict:
    """C = A*A on each stand-in: median of whole calls, GFLOP/s."""
    import torch
    from paper_2112_10037_amd import binding, gen
    rows = []
    for name, A in gen.table4_standins():
        prods = int(row_products(A, A).sum())
        dA = binding.DeviceCSR.from_host(A, "cuda:0")
        C = h.spgemm(dA, dA)
        nnz_c = C.nnz
        del C
        ts = step_times(h, dA, steps)
        h.sync()
        med = float(np.median(ts))
        rows.append({"name": name, "rows": A.nrows, "nnz_a": A.nnz, "products": prods, "nnz_c": nnz_c,
                     "ms": round(med * 1e3, 4), "gflops": round(2.0 * prods / med / 1e9, 3),
                     "paper_fpga_ms_context": PAPER_FPGA_MS[name]})
        del dA
        torch.cuda.empty_cache()
    return {"workload": "FP32 stand-ins of the paper's eight matrices (Table IV dimensions and densities), "
                        "C = A*A, plain path",
            "geomean_gflops": round(geomean([r["gflops"] for r in rows]), 3), "per_matrix": rows}


# ---------------------------------------------------------------------------
# host data (built before the GPU is touched: the pool forks)
# ---------------------------------------------------------------------------
def _build_member(m):
    return m.index, m.build()


def build_suite(workers: int):
    from concurrent.futures import ProcessPoolExecutor
    from paper_2112_10037_amd import gen
    suite = gen.learned_suite()
    mats = {}
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for i, M in ex.map(_build_member, suite):
            mats[i] = M
    return suite, mats


def timed(fn, reps: int):
    """Median wall time (s) of fn() over reps calls after one warm call; fn
    waits for its own result."""
    fn()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def geomean(x):
    return float(math.exp(np.mean(np.log(np.asarray(x, dtype=np.float64)))))


# ---------------------------------------------------------------------------
# legs
# ---------------------------------------------------------------------------
def learned_leg(h, suite, mats, reps: int, steps: int) -> dict:
    import torch
    from paper_2112_10037_amd import binding, learned
    dev = lambda M: binding.DeviceCSR.from_host(M, "cuda:0")          # noqa: E731
    t0 = time.perf_counter()
    train = [m for m in suite if not m.held_out]
    test = [m for m in suite if m.held_out]
    prods = []
    for m in train:
        d = dev(mats[m.index])
        prods.append((d, d))
    feats, targets = learned.training_set(h, prods)
    del prods
    t_rows = time.perf_counter() - t0
    progress(f"learned: {int(feats.shape[0])} training rows in {t_rows:.1f} s")
    t1 = time.perf_counter()
    pred, losses, delta = learned.train(h, feats, targets, steps=steps, batch=4096, seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    progress(f"learned: trained {steps} steps in {t_train:.1f} s, loss {losses[0]:.4f} -> {np.mean(losses[-20:]):.5f}")
    upper = binding.Predictor(h, learned.fixed_capacity_params(8.0))
    lin = binding.Predictor(h, learned.linear_fit_params(feats.cpu().numpy(), targets.cpu().numpy()))
    lin.calibrate(feats, targets, 0.99)
    n_train_rows = int(feats.shape[0])
    del feats, targets
    torch.cuda.empty_cache()

    rows = []
    for m in test:
        M = mats[m.index]
        dM = dev(M)

        def run_plain():
            C = h.spgemm(dM, dM)
            return C

        t_plain = timed(lambda: run_plain(), reps)
        Cp = run_plain()
        res = {"index": m.index, "family": m.family, "rows": M.nrows, "nnz_a": M.nnz,
               "nnz_c": Cp.nnz, "plain_ms": round(t_plain * 1e3, 3)}
        for name, p in (("learned", pred), ("network_free", upper), ("linear_fit", lin)):
            st = {}

            def run_l(p=p, st=st):
                C, s = h.spgemm_learned(p, dM, dM)
                st.update(s)
                return C

            t = timed(run_l, reps)
            C = run_l()
            same = bool(torch.equal(C.row_ptr, Cp.row_ptr) and torch.equal(C.col, Cp.col))
            res[name] = {"ms": round(t * 1e3, 3), "speedup": round(t_plain / t, 4),
                         "overflow_rows": st["overflow_rows"], "exact_rows": st["exact_rows"],
                         "sum_cap_over_nnz": round(st["sum_cap"] / max(Cp.nnz, 1), 4),
                         "structure_identical": same}
            del C
        del Cp, dM
        torch.cuda.empty_cache()
        rows.append(res)
        progress(f"learned: held-out {m.index} ({m.family}, {M.nrows} rows): plain {res['plain_ms']} ms, "
                 f"learned x{res['learned']['speedup']}, network-free x{res['network_free']['speedup']}")
    out = {"workload": "64-matrix mixed suite (27-point stencils n~U[41,101], ER 2^16..2^20 rows with 4..32 "
                       "nnz/row, R-MAT 2^16..2^18 rows with degree 8..32; FP64 U[-1,1]; seeds 1000+i), "
                       "C = A*A; trained on 48, evaluated on the 16 held out (index = 3 mod 4)",
           "training": {"rows": n_train_rows, "steps": steps, "batch": 4096,
                        "loss_first": round(float(losses[0]), 6), "loss_last": round(float(np.mean(losses[-20:])), 6),
                        "delta": round(float(delta), 4), "rows_s": round(t_rows, 2), "train_s": round(t_train, 2)}}
    for name in ("learned", "network_free", "linear_fit"):
        total_ovf = sum(r[name]["overflow_rows"] for r in rows)
        total_rows = sum(r["rows"] for r in rows)
        out[name] = {"geomean_speedup_vs_plain": round(geomean([r[name]["speedup"] for r in rows]), 4),
                     "overflow_rate": round(total_ovf / total_rows, 5),
                     "mean_sum_cap_over_nnz": round(float(np.mean([r[name]["sum_cap_over_nnz"] for r in rows])), 4),
                     "all_structure_identical": all(r[name]["structure_identical"] for r in rows)}
    out["per_matrix"] = rows
    for p in (pred, upper, lin):
        p.close()
    return out


def batched_leg(h, sides, reps: int, tuning_cache: str, meter=None) -> dict:
    import torch
    from paper_2112_10037_amd import batch, binding, gen
    t0 = time.perf_counter()
    pA, pP, pR = batch.galerkin_batch(sides)
    t_gen = time.perf_counter() - t0
    progress(f"batched: {len(sides)} problems packed and uploaded in {t_gen:.1f} s")
    # autotune on a seeded 32-problem subset, cached by the subset's shape
    sub = np.random.default_rng(5).choice(len(sides), 32, replace=False)
    sA, sP, sR = batch.galerkin_batch(sides[np.sort(sub)])
    tuning, tinfo = batch.autotune_cached(h, sA, sP, sR, tuning_cache)
    del sA, sP, sR
    t1 = time.perf_counter()
    plan = binding.Batch(h, pA, pP, pR, tuning=tuning)
    t_plan = time.perf_counter() - t1
    info = plan.info()
    progress(f"batched: tuning {tuning} (cached: {tinfo['cached']}), plan made in {t_plan:.1f} s")

    def replay():
        plan.execute()
        plan.sync()

    t_graph = timed(replay, reps)
    # the same plan with one static row range per wave instead of the work queue
    plan_s = binding.Batch(h, pA, pP, pR, tuning=tuning, queue_rows=-1)

    def replay_static():
        plan_s.execute()
        plan_s.sync()

    t_static = timed(replay_static, reps)
    plan_s.close()
    nprob = len(sides)
    energy = None
    if meter:
        energy = energy_entry(meter, replay, int(pA.nnz + int(info["nnz"][0])), "f64")

    def plain_all():
        for p in range(nprob):
            AP = h.spgemm(pA.view(p), pP.view(p), check=False)
            C = h.spgemm(pR.view(p), AP, check=False)
            del AP, C
        h.sync()
        torch.cuda.synchronize()

    progress(f"batched: graph replay {t_graph * 1e3:.2f} ms")
    t_plain = timed(plain_all, max(1, reps // 5))
    progress(f"batched: 1,024 plain calls {t_plain * 1e3:.1f} ms")
    # identical results (integer values) on a few problems
    same = True
    for p in (0, nprob // 2, nprob - 1):
        AP = h.spgemm(pA.view(p), pP.view(p))
        C = h.spgemm(pR.view(p), AP)
        Cb = plan.result(p)
        same = same and bool(torch.equal(C.row_ptr, Cb.row_ptr) and torch.equal(C.col, Cb.col)
                             and torch.equal(C.val, Cb.val))
    nnz_a, nnz_ap = pA.nnz, int(info["nnz"][0])
    nnz_ac = int(info["nnz"][1])
    products = nnz_a + nnz_ap      # P and R hold one entry per fine row
    m_a, m_ac = int(pA.row_start[-1]), int(pR.row_start[-1])
    alg = (csr_bytes(m_a, nnz_a) + csr_bytes(m_a, pP.nnz) + csr_bytes(m_a, nnz_ap)
           + csr_bytes(m_ac, pR.nnz) + csr_bytes(m_a, nnz_ap) + csr_bytes(m_ac, nnz_ac))
    plan.close()
    return {"workload": f"{nprob} Galerkin products R (A P), A = 3D 7-point Laplacian n^3 (n ~ U{{16..64}}, "
                        f"seed 5), P = 2x2x2 aggregation, FP64",
            "rows_fine": m_a, "rows_coarse": m_ac, "nnz_a": nnz_a, "nnz_ap": nnz_ap, "nnz_ac": nnz_ac,
            "products": products, "graph_ms": round(t_graph * 1e3, 3),
            "graph_ms_static_split": round(t_static * 1e3, 3), "work_queue_rows": 1024,
            "plain_1024_calls_ms": round(t_plain * 1e3, 3),
            "speedup": round(t_plain / t_graph, 3),
            "graph_gflops": round(2 * products / t_graph / 1e9, 3),
            "plain_gflops": round(2 * products / t_plain / 1e9, 3),
            "graph_algorithmic_gbs": round(alg / t_graph / 1e9, 1),
            "tuning": list(tuning), "tuning_cached": tinfo["cached"],
            "autotune_median_ms": tinfo.get("median_ms"),
            "plan": info, "plan_s": round(t_plan, 2), "generate_s": round(t_gen, 2),
            "results_identical_to_plain": same, "energy": energy}


OMAR_GROUPS = (2, 4, 8, 16, 32, 64)


def sharing_leg(h, dmain, main_name: str, mats, reps: int = 20) -> dict:
    """B-row sharing (Sec. IV-A): OMAR of Eq. (1) at the paper's group sizes
    on each config (computed on the GPU), and the numeric merge with and
    without the LDS stage on the 2D Laplacian and on a Galerkin A P (n = 32)."""
    import torch
    from paper_2112_10037_amd import binding, gen
    out = {"omar_percent": {}, "groups": list(OMAR_GROUPS)}

    def omar_row(dX):
        return [round(h.omar(dX, g), 3) for g in OMAR_GROUPS]

    for name in ("er4096", "laplacian2d_1024"):
        _, X = workload(name)
        dX = binding.DeviceCSR.from_host(X, "cuda:0")
        out["omar_percent"][name] = omar_row(dX)
        del dX
    out["omar_percent"][main_name] = omar_row(dmain)
    if mats is not None:
        for i in (11, 15, 7):                # one suite member per family
            dX = binding.DeviceCSR.from_host(mats[i], "cuda:0")
            out["omar_percent"][f"suite_{i}_{('er', 'rmat', 'stencil27')[i % 3]}"] = omar_row(dX)
            del dX

    def timing(X, Y, base, label):
        dX = binding.DeviceCSR.from_host(X, "cuda:0")
        dY = dX if Y is X else binding.DeviceCSR.from_host(Y, "cuda:0")
        res = {}
        for g in (0, 16, 32, 64):
            t = tuple(base) + ((g,) if g else ())
            C = h.spgemm(dX, dY, tuning=t)
            del C
            h.sync()
            h.profile(True, phases=["numeric"])
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                C = h.spgemm(dX, dY, tuning=t, check=False)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                del C
            h.sync()
            num_ms, num_n = h.profile_get()["numeric"]
            h.profile(False)
            st = h.share_stats()
            key = f"share_g_{g}" if g else "unshared"
            res[key] = {"ms_median": round(float(np.median(ts)) * 1e3, 4),
                        "numeric_ms": round(num_ms / max(num_n, 1), 5)}
            if g:
                res[key].update(st)
                if st["a_entries"]:
                    res[key]["b_reads_saved_percent"] = round(
                        100.0 * (st["a_entries"] - st["b_rows"]) / st["a_entries"], 3)
        del dX, dY
        torch.cuda.empty_cache()
        progress(f"sharing: {label}: " + ", ".join(f"{k} {v['numeric_ms']} ms" for k, v in res.items()))
        return res

    _, L = workload("laplacian2d_1024")
    out["laplacian2d_1024_numeric"] = timing(L, L, (1, 0, 4096, 1024, 8), "laplacian2d_1024")
    # (a 3D band spans 2 n^2 B rows: n = 32 keeps a batch within the stage's
    # 4,096-row span bitmap)
    A, P, _ = gen.galerkin_problem(32)
    out["galerkin32_AP_numeric"] = timing(A, P, (1, 0, 4096, 1024, 8), "galerkin n=32, A P")
    return out


# plain-path tunings the autotuner compares on the main workload
PLAIN_CANDIDATES = [(1, 0, 4096, 1024, 8), (1, 0, 2048, 1024, 8), (1, 0, 1024, 1024, 8), (2, 0, 4096, 1024, 8)]


def autotune_plain(h, dA, A, path: str, candidates=PLAIN_CANDIDATES, reps: int = 3):
    """Best plain-path tuning for this product's shape: from the JSON cache
    at `path` when it holds one, else measured with msp_autotune (median of
    whole calls) and stored.  Returns (tuning, info)."""
    key = "plain:" + hashlib.sha256(np.ascontiguousarray(A.row_ptr).tobytes()[:1 << 20] +
                                    str((A.nrows, A.ncols, A.nnz, str(A.val.dtype))).encode()).hexdigest()[:24]
    cache = {}
    if path and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        return tuple(cache[key]["tuning"]), {"cached": True, "median_ms": cache[key].get("median_ms")}
    best, times = h.autotune(dA, dA, candidates, reps=reps)
    cache[key] = {"tuning": list(best), "candidates": [list(c) for c in candidates],
                  "median_ms": [round(t, 3) for t in times]}
    if path:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return tuple(best), {"cached": False, "median_ms": cache[key]["median_ms"]}


def step_times(h, dA, steps: int):
    """Seconds of each of `steps` whole calls, each waited for."""
    import torch
    ts = []
    for _ in range(steps):
        t0 = time.perf_counter()
        C = h.spgemm(dA, dA, check=False)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        del C
    return ts


def config_entry(h, name: str, steps: int, warmup: int) -> dict:
    """One of the smaller configs timed like the main line (median of whole
    calls), with its numeric phase's algorithmic rate."""
    import torch
    from paper_2112_10037_amd import binding
    desc, A = workload(name)
    prods = int(row_products(A, A).sum())
    dA = binding.DeviceCSR.from_host(A, "cuda:0")
    C = h.spgemm(dA, dA)
    nnz_c = C.nnz
    del C
    for _ in range(warmup):
        C = h.spgemm(dA, dA)
        del C
    h.sync()
    h.profile(True, phases=["numeric"])
    ts = step_times(h, dA, steps)
    h.sync()
    num_ms, num_n = h.profile_get()["numeric"]
    h.profile(False)
    med = float(np.median(ts))
    num_s = num_ms / max(num_n, 1) / 1e3
    alg = algorithmic_bytes(A, nnz_c)
    del dA
    torch.cuda.empty_cache()
    return {"workload": desc, "rows": A.nrows, "nnz_a": A.nnz, "products": prods, "nnz_c": nnz_c,
            "steps": steps, "ms_per_step_median": round(med * 1e3, 4),
            "gflops": round(2.0 * prods / med / 1e9, 3),
            "numeric_ms": round(num_s * 1e3, 5),
            "numeric_algorithmic_gbs": round(alg / num_s / 1e9, 1),
            "numeric_frac_of_peak": round(alg / num_s / 1e9 / HBM_PEAK_GBS, 4)}


def global_bin_bytes(A, row_nnz: np.ndarray, thresh: int) -> tuple[int, int]:
    """Algorithmic bytes of one launch of the global bin's kernel: for each
    row with more than `thresh` outputs, its A row (8 B of row pointers and
    one column and value per entry), its C row (the same), and B once
    (every row pointer and entry).  Returns (bytes, rows)."""
    vb = A.val.dtype.itemsize
    g = row_nnz > thresh
    nnz_a = np.diff(A.row_ptr)
    b = (A.nrows + 1) * 8 + A.nnz * (4 + vb)
    per_row = int(g.sum()) * 16 + int(nnz_a[g].sum()) * (4 + vb) + int(row_nnz[g].sum()) * (4 + vb)
    return per_row + b, int(g.sum())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat20")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the smaller configs' entries")
    ap.add_argument("--no-energy", action="store_true", help="skip the energy entries")
    ap.add_argument("--no-table4", action="store_true", help="skip the Table IV stand-ins")
    ap.add_argument("--no-sharing", action="store_true", help="skip the B-row sharing leg (OMAR, staged merge)")
    ap.add_argument("--no-autotune", action="store_true", help="run the library's default tuning")
    ap.add_argument("--legs-reps", type=int, default=5)
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--tuning-cache", default=os.path.join(os.path.expanduser("~"), ".cache", "msp_tuning.json"))
    ap.add_argument("--tuning", default=None,
                    help="hash_scale,group_scale,spill_nnz,block_rows,merge_k (default: autotuned)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--vendor", action="store_true",
                    help="also time the same product through torch.sparse.mm (hipSPARSE), as context")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path in this library "
              "(the design notes describe how the product would shard).", file=sys.stderr)
        sys.exit(2)

    from paper_2112_10037_amd import gen
    t0 = time.perf_counter()
    desc, A = workload(args.workload)
    prods_row = row_products(A, A)
    products = int(prods_row.sum())
    progress(f"main workload built in {time.perf_counter() - t0:.1f} s")
    workers = max(1, min(16, os.cpu_count() or 1))
    suite = mats = None
    if not args.no_learned:
        t0 = time.perf_counter()
        suite, mats = build_suite(workers)
        progress(f"suite of {len(mats)} matrices built in {time.perf_counter() - t0:.1f} s")
    sides = gen.galerkin_sizes(512, 16, 64, seed=5)

    import torch
    from paper_2112_10037_amd import binding

    dA = binding.DeviceCSR.from_host(A, "cuda:0")
    h = binding.Handle(0)
    tinfo = None
    if args.tuning:
        h.set_tuning(tuple(int(x) for x in args.tuning.split(",")))
    elif not args.no_autotune:
        tuning, tinfo = autotune_plain(h, dA, A, args.tuning_cache)
        h.set_tuning(tuning)
        progress(f"plain tuning {tuning} (cached: {tinfo['cached']})")
    tuning = h.get_tuning()

    # the cold first call (workspace allocations, first launches), reported apart
    torch.cuda.synchronize()
    t_cold = time.perf_counter()
    C = h.spgemm(dA, dA)
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t_cold) * 1e3
    nnz_c = C.nnz
    row_nnz = np.diff(C.row_ptr.cpu().numpy())
    del C
    for _ in range(args.warmup):
        C = h.spgemm(dA, dA)
        del C
    h.sync()

    # timed steps: HIP events around the global bin's kernel only (the
    # roofline's kernel), so that the rest runs as it does unprofiled
    h.profile(True, phases=["global_bin"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ts = step_times(h, dA, args.steps)
    el = time.perf_counter() - t0
    h.sync()          # raises if any timed call flagged an internal error
    prof = h.profile_get()
    # phase breakdown from a separate, fully profiled run
    h.profile(True)
    nph = max(3, args.steps // 3)
    for _ in range(nph):
        C = h.spgemm(dA, dA, check=False)
        del C
    h.sync()
    prof_all = h.profile_get()
    h.profile(False)

    med = float(np.median(ts))
    gflops = 2.0 * products / med / 1e9
    alg = algorithmic_bytes(A, nnz_c)
    gb_ms, gb_n = prof["global_bin"]
    roof = None
    if gb_n:
        gb_s = gb_ms / gb_n / 1e3
        gbytes, grows = global_bin_bytes(A, row_nnz, int(tuning[2]))
        achieved = gbytes / gb_s / 1e9
        key = MEASURED_TRAFFIC.get((args.workload, tuple(int(x) for x in tuning)))
        traffic = key["bytes"] if key and key["sources_sha256"] == kernel_sources_hash(tuning) else None
        roof = {"bound": "hbm", "kernel": "global bin, windowed numeric kernel (k_num_win)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes": gbytes, "rows": grows, "avg_launch_ms": round(gb_s * 1e3, 4),
                "launches_timed": gb_n}
    copy_gbs = copy_bandwidth()
    if roof:
        roof["copy_gbs"] = round(copy_gbs, 1)
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)
    vendor = vendor_spgemm(dA, products, nnz_c) if args.vendor else None

    out = {
        "metric": "SpGEMM GFLOP/s (2x products/s)",
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(med * 1e3, 4),
        "ms_per_step_mean": round(el * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if A.val.dtype == np.float64 else "f32",
        "data": "synthetic",
        "config": {"workload": desc, "rows": A.nrows, "nnz_a": A.nnz, "products": products,
                   "nnz_c": nnz_c, "path": "plain two-phase", "tuning": list(tuning),
                   "tuning_autotuned": tinfo},
        "roofline": roof,
        "hbm_gbs_whole_step_algorithmic": round(alg / med / 1e9, 1),
        "whole_step_frac_of_peak": round(alg / med / 1e9 / HBM_PEAK_GBS, 4),
        "first_call_ms": round(first_ms, 3),
        "phases_ms_per_step_profiled": {k: round(v[0] / nph, 4) for k, v in prof_all.items() if v[1]},
        "summary_fallbacks": h.summary_fallbacks(),
    }
    if vendor is not None:
        out["vendor_library"] = vendor
    meter = None
    if not args.no_energy:
        try:
            meter = EnergyMeter()
        except Exception as e:          # no SMI access on this machine
            out["energy"] = {"error": repr(e)[:200]}
    if meter:
        def one_call():
            C = h.spgemm(dA, dA, check=False)
            torch.cuda.synchronize()
            del C
        out["energy"] = energy_entry(meter, one_call, products, out["dtype"])
        progress(f"main: {out['energy']['joules_per_call']} J per SpGEMM")
    del dA
    torch.cuda.empty_cache()
    progress(f"main: {gflops:.1f} GFLOP/s, {med * 1e3:.3f} ms per step (median)")
    h.set_tuning((0, 0, 0, 0, 0))               # the library's defaults for the other legs
    if not args.no_configs:
        out["configs"] = {"er4096": config_entry(h, "er4096", 200, 10),
                          "laplacian2d_1024": config_entry(h, "laplacian2d_1024", 50, 5)}
        if meter:
            from paper_2112_10037_amd import binding as _b
            _, L = workload("laplacian2d_1024")
            dL = _b.DeviceCSR.from_host(L, "cuda:0")

            def lap_call():
                C = h.spgemm(dL, dL, check=False)
                torch.cuda.synchronize()
                del C
            out["configs"]["laplacian2d_1024"]["energy"] = energy_entry(
                meter, lap_call, out["configs"]["laplacian2d_1024"]["products"], "f64")
            del dL
        progress("configs done")
    if not args.no_sharing:
        dA = binding.DeviceCSR.from_host(A, "cuda:0")
        out["b_row_sharing"] = sharing_leg(h, dA, args.workload, mats)
        del dA
        torch.cuda.empty_cache()
    if not args.no_table4:
        out["table4_standins"] = table4_leg(h)
        progress(f"table4 stand-ins: geomean {out['table4_standins']['geomean_gflops']} GFLOP/s")
    if not args.no_learned:
        out["learned_vs_plain"] = learned_leg(h, suite, mats, args.legs_reps, args.train_steps)
        del mats
    if not args.no_batched:
        out["batched_vs_plain"] = batched_leg(h, sides, max(args.legs_reps, 10), args.tuning_cache, meter)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(A, prods_row, args.cpu_seconds)
    if meter:
        meter.close()
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
