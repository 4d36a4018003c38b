"""The allocation-free entry point (msp_spgemm_noalloc) against msp_spgemm
through the C ABI: identical structure, values within the oracle's bound
of each other and of the oracle, on two calls in a row (the second on a
smaller input, so that the shared scratch holds the first call's data);
too small a capacity and too many rows are refused cleanly."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2112_10037_amd import binding, gen

from gpu_util import TOL, long_rows_case, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(h, A, B, capacity):
    import torch
    dA, dB = to_dev(A), to_dev(B)
    vdt = torch.float64 if A.val.dtype == np.float64 else torch.float32
    rp = torch.empty(A.nrows + 1, dtype=torch.int64, device="cuda")
    col = torch.full((max(capacity, 1),), -7, dtype=torch.int32, device="cuda")
    val = torch.zeros(max(capacity, 1), dtype=vdt, device="cuda")
    out = binding.c_csr_out()
    out.row_ptr, out.col, out.val = rp.data_ptr(), col.data_ptr(), val.data_ptr()
    a, b = dA.c(), dB.c()
    st = h._lib.msp_spgemm_noalloc(h._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(out), capacity, None)
    torch.cuda.synchronize()
    return st, out, rp, col, val


def _check_against_plain(h, A, B):
    import torch
    ref = h.spgemm(to_dev(A), to_dev(B)).to_host()
    before = len(h._live)
    st, out, rp, col, val = _noalloc(h, A, B, ref.nnz + 17)
    assert binding.STATUS[st] == "MSP_OK", h._lib.msp_last_error()
    h.sync()
    assert len(h._live) == before                     # the allocator was not called
    n = int(out.nnz)
    assert n == ref.nnz and out.col == col.data_ptr() and out.val == val.data_ptr()
    got_rp, got_col, got_val = rp.cpu().numpy(), col[:n].cpu().numpy(), val[:n].cpu().numpy()
    assert np.array_equal(got_rp, ref.row_ptr) and np.array_equal(got_col, ref.col)
    assert np.all(col[n:].cpu().numpy() == -7)        # nothing written past nnz(C)
    o = oracle.spgemm(A, B)
    tol = TOL[np.dtype(A.val.dtype)]
    oracle.compare(got_rp, got_col, got_val, o, tol)
    # and within the bound of the plain entry point's values
    assert np.all(np.abs(got_val - ref.val) <= 2 * tol * o[3])


def test_noalloc_matches_plain_twice():
    h = binding.Handle(0)
    try:
        big = gen.rmat(12, 16 << 12, seed=51, dtype=np.float64)       # hash and global bins
        _check_against_plain(h, big, big)
        small = gen.erdos_renyi(700, 900, 6, seed=52)
        B = gen.erdos_renyi(900, 500, 5, seed=53)
        _check_against_plain(h, small, B)
        wide = gen.erdos_renyi(300, 4000, 20, seed=54, dtype=np.float32)
        W = gen.erdos_renyi(4000, 1 << 19, 300, seed=55, dtype=np.float32)   # windowed global bin
        _check_against_plain(h, wide, W)
        _check_against_plain(h, small, B)
    finally:
        h.close()


def test_noalloc_first_call_on_fresh_handle():
    """The allocation-free product as a fresh handle's first call, on rows
    with more than 256 A entries (the statistics pass's long-row lists)
    and on a skewed matrix: every workspace it touches must come from the
    scratch array, since the library refuses any other workspace growth
    during this call as an internal error.  Then the plain product, and the
    allocation-free one again on a smaller input."""
    for A, B in (long_rows_case(), (gen.rmat(12, 16 << 12, seed=57),) * 2):
        h = binding.Handle(0)
        try:
            o = oracle.spgemm(A, B)
            st, out, rp, col, val = _noalloc(h, A, B, int(o[0][-1]))
            assert binding.STATUS[st] == "MSP_OK", h._lib.msp_last_error()
            n = int(out.nnz)
            oracle.compare(rp.cpu().numpy(), col[:n].cpu().numpy(), val[:n].cpu().numpy(), o,
                           TOL[np.dtype(A.val.dtype)])
            _check_against_plain(h, A, B)
            small = gen.erdos_renyi(300, A.ncols, 3, seed=58, dtype=A.val.dtype)
            _check_against_plain(h, small, B)
        finally:
            h.close()


def test_noalloc_refuses_cleanly():
    h = binding.Handle(0)
    try:
        A = gen.erdos_renyi(500, 500, 6, seed=56)
        ref = oracle.spgemm(A, A)
        need = int(ref[0][-1])
        st, out, rp, col, val = _noalloc(h, A, A, need - 1)
        assert binding.STATUS[st] == "MSP_ERR_INVALID_ARG"
        assert int(out.nnz) == need and b"capacity" in h._lib.msp_last_error()
        assert np.array_equal(rp.cpu().numpy(), ref[0])          # the row pointers are there
        assert np.all(col.cpu().numpy() == -7)                     # no entry written
        h.sync()
        # too many rows for the scratch: refused before anything runs
        big = binding.c_csr(8 << 20, 500, 0, rp.data_ptr(), None, None, binding.MSP_F64)
        a = to_dev(gen.erdos_renyi(500, 500, 6, seed=56)).c()
        o = binding.c_csr_out()
        o.row_ptr = rp.data_ptr()
        st = h._lib.msp_spgemm_noalloc(h._h, ctypes.byref(big), ctypes.byref(a), ctypes.byref(o), 0, None)
        assert binding.STATUS[st] == "MSP_ERR_INVALID_ARG" and b"rows exceed" in h._lib.msp_last_error()
        # the handle still works
        st, out, rp, col, val = _noalloc(h, A, A, need)
        assert binding.STATUS[st] == "MSP_OK"
        oracle.compare(rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy(), ref, 1e-12)
    finally:
        h.close()
