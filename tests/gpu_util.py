"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare with the CPU oracle."""
import numpy as np

import oracle
from paper_2112_10037_amd import binding, gen

TOL = {np.dtype(np.float64): 1e-12, np.dtype(np.float32): 1e-5}


def to_dev(m):
    return binding.DeviceCSR.from_host(m)


def run(h, A, B, **kw):
    import torch
    C = h.spgemm(to_dev(A), to_dev(B), **kw)
    torch.cuda.synchronize()
    return C


def check_full(h, A, B, **kw):
    """Whole-matrix parity: identical structure, values within the bound."""
    C = run(h, A, B, **kw)
    ref = oracle.spgemm(A, B)
    host = C.to_host()
    assert host.val.dtype == A.val.dtype
    return oracle.compare(host.row_ptr, host.col, host.val, ref, TOL[np.dtype(A.val.dtype)])


def check_rows(C, A, B, rows):
    """Parity on sampled rows of a device result (oracle row by row)."""
    import torch
    rp = C.row_ptr
    tol = TOL[np.dtype(A.val.dtype)]
    worst = 0.0
    for r in rows:
        r = int(r)
        ref = oracle.spgemm(A, B, r, r + 1)
        s, e = int(rp[r].item()), int(rp[r + 1].item())
        col = C.col[s:e].cpu().numpy()
        val = C.val[s:e].cpu().numpy()
        worst = max(worst, oracle.compare(np.array([0, e - s]), col, val, ref, tol))
    return worst


def long_rows_case(dtype=np.float64):
    """1,000 rows of A over 30,000 columns: most with 0..8 entries, rows 5
    and 77 with 20,000, row 640 with 6,000, and row 300 with 5,000 entries
    that select only empty B rows (B rows 25,000 on are empty)."""
    rng = np.random.default_rng(71)
    m, k, n = 1000, 30_000, 2000
    rows = []
    for i in range(m):
        if i in (5, 77):
            c = rng.choice(k, 20_000, replace=False)
        elif i == 640:
            c = rng.choice(k, 6_000, replace=False)
        elif i == 300:
            c = 25_000 + rng.choice(5_000, 5_000, replace=False)
        else:
            c = rng.choice(k, int(rng.integers(0, 9)), replace=False)
        rows.append(np.sort(c))
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    A = gen.CSR(m, k, rp, np.concatenate(rows).astype(np.int32), rng.uniform(-1, 1, int(rp[-1])).astype(dtype))
    kb = rng.integers(0, 6, k)
    kb[25_000:] = 0
    B = gen.erdos_renyi(k, n, kb, seed=72, dtype=dtype)
    return A, B
