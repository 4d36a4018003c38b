"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare with the CPU oracle."""
import numpy as np

import oracle
from paper_2112_10037_amd import binding

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
