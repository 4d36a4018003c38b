"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Structure (row_ptr, col) must be identical; values must satisfy
|c - o| <= tol * sum_k |a_ik||b_kj| with tol 1e-12 (FP64) or 1e-5 (FP32).
"""
import ctypes
import json
import os

import numpy as np
import pytest

import oracle
from paper_2112_10037_amd import binding, gen

from gpu_util import TOL, check_full, check_rows, long_rows_case, run, to_dev

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hh = binding.Handle(0)
    yield hh
    hh.close()


def _rand(rng, m, k, density, dtype=np.float64):
    pat = rng.random((m, k)) < density
    return gen.from_dense(np.where(pat, rng.uniform(-1, 1, (m, k)), 0.0).astype(dtype), pattern=pat)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_hand_products(h, dtype):
    cases = json.load(open(os.path.join(GOLDEN, "hand_products.json")))["cases"]
    for c in cases:
        d = c["A"]
        A = gen.CSR(d["nrows"], d["ncols"], np.array(d["row_ptr"], np.int64),
                    np.array(d["col"], np.int32), np.array(d["val"], dtype))
        if c["B"] == "A":
            B = A
        else:
            d = c["B"]
            B = gen.CSR(d["nrows"], d["ncols"], np.array(d["row_ptr"], np.int64),
                        np.array(d["col"], np.int32), np.array(d["val"], dtype))
        C = run(h, A, B).to_host()
        assert C.row_ptr.tolist() == c["C"]["row_ptr"], c["name"]
        assert C.col.tolist() == c["C"]["col"], c["name"]
        assert C.val.tolist() == [float(v) for v in c["C"]["val"]], c["name"]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_dense_tiny(h, seed, dtype):
    rng = np.random.default_rng(seed)
    m, k, n = (int(x) for x in rng.integers(1, 49, 3))
    A = _rand(rng, m, k, rng.uniform(0, 0.6), dtype)
    B = _rand(rng, k, n, rng.uniform(0, 0.6), dtype)
    check_full(h, A, B)


def test_er_4096_exact8(h):
    """ER 4096 x 4096, exactly 8 nonzeros per row, FP64, seed 0 (C = A*A)."""
    A = gen.erdos_renyi(4096, 4096, 8, seed=0)
    err = check_full(h, A, A)
    print(f"max |c-o|/bound = {err:.3e}")


def test_laplacian_2d_1024_exact(h):
    """2D 5-point Laplacian on 1024^2, FP64: every value is a small integer, so
    the GPU sums must equal the oracle's bit for bit."""
    A = gen.laplacian_2d(1024)
    C = run(h, A, A).to_host()
    rp, col, val, bnd = oracle.spgemm(A, A)
    assert np.array_equal(C.row_ptr, rp) and np.array_equal(C.col, col)
    assert np.array_equal(C.val, val)
    assert C.nnz == 13_611_012


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("scale", [10, 13])
def test_rmat_skewed(h, scale, dtype):
    A = gen.rmat(scale, 16 << scale, seed=3, dtype=dtype)
    check_full(h, A, A)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_forced_spill(h, dtype):
    A = gen.rmat(11, 16 << 11, seed=5, dtype=dtype)
    check_full(h, A, A, force_spill=True)
    B = gen.erdos_renyi(3000, 3000, 7, seed=2, dtype=dtype)
    check_full(h, B, B, force_spill=True)


def test_hub_rows_lds_bitmap_and_global_bin(h):
    """A few rows whose union exceeds every LDS table: symbolic bitmap (LDS)
    and the numeric global bin (column-window slices)."""
    rng = np.random.default_rng(8)
    n = 20000
    B = gen.erdos_renyi(n, n, 8, seed=9)
    k = np.full(40, 3, dtype=np.int64)
    k[[0, 7, 39]] = [3000, 6000, 1500]
    A = gen.erdos_renyi(40, n, k, seed=10)
    check_full(h, A, B)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_global_bin_many_slices(h, dtype):
    """2^19 columns: the row bitmap and its rank table take 72 KB of LDS, and
    rows of about 360,000 outputs are accumulated in LDS over about twenty
    column slices each, every slice found by a binary search in each B row."""
    n = 1 << 19
    B = gen.erdos_renyi(4096, n, 300, seed=21, dtype=dtype)
    k = np.full(32, 5, dtype=np.int64)
    k[[0, 13, 31]] = [2000, 1200, 2000]
    A = gen.erdos_renyi(32, 4096, k, seed=22, dtype=dtype)
    check_full(h, A, B)


@pytest.mark.parametrize("n,dtype", [(1 << 21, np.float64), ((1 << 21) + 12345, np.float32)])
def test_wide_matrix_global_bitmap(h, n, dtype):
    """ncols above 2^21: the n-bit bitmap no longer fits LDS.  The symbolic
    pass uses global bitmap slabs; the numeric pass walks two column
    super-ranges, each with its own LDS bitmap and slices (rows of 900 A
    entries keep their cursors, rows of 2500 search in every slice)."""
    B = gen.erdos_renyi(4000, n, 60, seed=11, dtype=dtype)
    k = np.full(16, 5, dtype=np.int64)
    k[[1, 9]] = [900, 2500]
    A = gen.erdos_renyi(16, 4000, k, seed=12, dtype=dtype)
    check_full(h, A, B)


def test_degenerate_shapes(h):
    import torch
    for (m, k, n) in [(0, 0, 0), (0, 5, 3), (4, 0, 3), (4, 5, 0), (3, 3, 3)]:
        A = gen.empty(m, k)
        B = gen.empty(k, n)
        C = run(h, A, B)
        assert C.nnz == 0 and C.row_ptr.cpu().tolist() == [0] * (m + 1)
    # one column, one row, empty rows mixed in
    A = gen.from_dense(np.ones((5, 1)))
    B = gen.from_dense(np.full((1, 1), 2.0))
    check_full(h, A, B)
    A = gen.from_dense(np.array([[0, 0, 0], [1.0, 0, 2], [0, 0, 0]]))
    check_full(h, A, A)


def test_all_zero_values_keep_structure(h):
    A = gen.erdos_renyi(500, 500, 6, seed=4)
    A.val[:] = 0.0
    C = run(h, A, A).to_host()
    rp, col, _, _ = oracle.spgemm(A, A)
    assert np.array_equal(C.row_ptr, rp) and np.array_equal(C.col, col)
    assert np.all(C.val == 0.0)


def test_hash_hostile_columns(h):
    """Columns that are all multiples of 4096 (congruent mod every table size)."""
    n = 1 << 22
    rng = np.random.default_rng(6)
    rows = 300
    k = rng.integers(1, 60, rows)
    cols = [np.sort(rng.choice(n // 4096, size=int(x), replace=False)) * 4096 for x in k]
    rp = np.zeros(rows + 1, np.int64)
    np.cumsum(k, out=rp[1:])
    B = gen.CSR(rows, n, rp, np.concatenate(cols).astype(np.int32), rng.uniform(-1, 1, int(rp[-1])))
    A = gen.erdos_renyi(200, rows, 12, seed=7)
    check_full(h, A, B)


@pytest.mark.parametrize("merge_k", [4, 8])
def test_merge_rows_with_many_entries_fall_back(h, merge_k):
    """Rows in the merge bin with more A entries than merge_k take the wave
    fallback; mixed with rows that merge."""
    n = 64
    k = np.random.default_rng(3).integers(1, 12, 3000)
    A = gen.erdos_renyi(3000, n, k, seed=31)
    B = gen.erdos_renyi(n, 2000, 1, seed=32)
    check_full(h, A, B, tuning=(1, 0, 4096, 128, merge_k))
    C = gen.erdos_renyi(3000, 3000, 5, seed=33, dtype=np.float32)
    check_full(h, C, C, tuning=(1, 0, 4096, 128, merge_k))


def test_rectangular_chain(h):
    rng = np.random.default_rng(21)
    A = _rand(rng, 300, 700, 0.02)
    B = _rand(rng, 700, 90, 0.05)
    check_full(h, A, B)


def test_transpose_identity_structure(h):
    import scipy.sparse as sp
    A = gen.rmat(10, 8 << 10, seed=13, dtype=np.float64)
    B = gen.erdos_renyi(1024, 1024, 5, seed=14)

    def T(M):
        s = sp.csr_matrix((M.val, M.col, M.row_ptr), shape=(M.nrows, M.ncols)).T.tocsr()
        s.sort_indices()
        return gen.CSR(M.ncols, M.nrows, s.indptr.astype(np.int64), s.indices.astype(np.int32), s.data)

    C = run(h, A, B).to_host()
    Ct = run(h, T(B), T(A)).to_host()
    CT = T(C)
    assert np.array_equal(CT.row_ptr, Ct.row_ptr) and np.array_equal(CT.col, Ct.col)
    ref = oracle.spgemm(T(B), T(A))
    oracle.compare(Ct.row_ptr, Ct.col, Ct.val, ref, 1e-12)


TUNINGS = [(1, 0, 4096, 128, 8), (2, 0, 4096, 128, 4), (1, 1, 1024, 64, -1), (2, 2, 256, 32, 8),
           (1, 2, 512, 128, -1), (2, 1, 2048, 128, 4), (1, 0, 4096, 1024, 8), (2, 0, 4096, 1024, 8),
           (1, 1, 2048, 512, -1), (2, 2, 1024, 256, 4)]


@pytest.mark.parametrize("tuning", TUNINGS)
def test_tuning_variants_same_result(h, tuning):
    A = gen.rmat(12, 12 << 12, seed=15, dtype=np.float64)
    check_full(h, A, A, tuning=tuning)


@pytest.mark.parametrize("tuning", [(1, 0, 4096, 128, 8), (1, 0, 4096, 1024, 8), (2, 0, 4096, 1024, 8),
                                    (1, 1, 512, 256, -1)])
def test_stencil27_bins(h, tuning):
    """27-point rows: 729 products, 125 outputs (one-wave tables up to 1024
    bounds, or workgroups)."""
    A = gen.stencil_27(14, seed=16, dtype=np.float64)
    check_full(h, A, A, tuning=tuning)


def test_validation_errors(h):
    A = gen.erdos_renyi(50, 50, 4, seed=1)
    bad = gen.CSR(A.nrows, A.ncols, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    bad.col[1], bad.col[2] = bad.col[2], bad.col[1]       # unsorted row 0
    with pytest.raises(binding.MspError) as e:
        h.spgemm(to_dev(bad), to_dev(A), validate=True)
    assert e.value.name == "MSP_ERR_UNSORTED_OR_DUP"
    oor = gen.CSR(A.nrows, A.ncols, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    oor.col[-1] = 50                                      # out of range
    with pytest.raises(binding.MspError) as e:
        h.spgemm(to_dev(oor), to_dev(A), validate=True)
    assert e.value.name == "MSP_ERR_INVALID_ARG"
    B = gen.erdos_renyi(40, 40, 4, seed=2)
    with pytest.raises(binding.MspError) as e:
        h.spgemm(to_dev(A), to_dev(B))
    assert e.value.name == "MSP_ERR_SHAPE"
    with pytest.raises(binding.MspError) as e:
        h.spgemm(to_dev(A), to_dev(A.astype(np.float32)))
    assert e.value.name == "MSP_ERR_DTYPE"
    # more rows than the launch grids can be rounded up from: refused before
    # anything is read (the row_ptr given is far too short on purpose)
    dA = to_dev(A)
    big = binding.c_csr(2**31 - 8192, 50, 0, dA.row_ptr.data_ptr(), None, None, binding.MSP_F64)
    a = dA.c()
    out = binding.c_csr_out()
    st = h._lib.msp_spgemm(h._h, ctypes.byref(big), ctypes.byref(a), ctypes.byref(out), None)
    assert binding.STATUS[st] == "MSP_ERR_INDEX_OVERFLOW"
    check_full(h, A, A, validate=True)


def test_symbolic_and_features(h):
    A = gen.rmat(12, 16 << 12, seed=17, dtype=np.float64)
    dA = to_dev(A)
    rn, tot = h.symbolic(dA, dA)
    ref = oracle.row_nnz(A, A)
    assert np.array_equal(rn.cpu().numpy(), ref) and tot == ref.sum()
    prod, feat = h.row_features(dA, dA)
    st = oracle.row_stats(A, A)
    assert np.array_equal(prod.cpu().numpy(), st["prod"])
    f_ref = oracle.features(A, A)
    assert np.allclose(feat.cpu().numpy(), f_ref, rtol=2e-6, atol=2e-6)


def test_repeat_calls_deterministic_structure(h):
    A = gen.rmat(12, 16 << 12, seed=19, dtype=np.float32)
    dA = to_dev(A)
    C1 = h.spgemm(dA, dA)
    C2 = h.spgemm(dA, dA)
    import torch
    assert torch.equal(C1.row_ptr, C2.row_ptr) and torch.equal(C1.col, C2.col)


def _row_subset(M, rows):
    """The rows `rows` of M as a CSR matrix of their own (same columns)."""
    rp = M.row_ptr
    lens = rp[rows + 1] - rp[rows]
    nrp = np.zeros(rows.size + 1, np.int64)
    np.cumsum(lens, out=nrp[1:])
    idx = np.repeat(rp[rows] - nrp[:-1], lens) + np.arange(int(nrp[-1]))
    return gen.CSR(int(rows.size), M.ncols, nrp, M.col[idx], M.val[idx])


def _device_rows(C, rows):
    """(row_ptr from 0, col, val) on the host of the rows `rows` of a device
    result, gathered on the device."""
    import torch
    rp = C.row_ptr
    r = torch.from_numpy(rows.astype(np.int64)).to(rp.device)
    starts, lens = rp[r], rp[r + 1] - rp[r]
    nrp = torch.zeros(rows.size + 1, dtype=torch.int64, device=rp.device)
    torch.cumsum(lens, 0, out=nrp[1:])
    idx = torch.repeat_interleave(starts - nrp[:-1], lens) + torch.arange(int(nrp[-1]), device=rp.device)
    return nrp.cpu().numpy(), C.col[idx].cpu().numpy(), C.val[idx].cpu().numpy()


# numeric bins of the default tuning: exact row nnz in (lo, hi]
NUM_BIN_EDGES = [0, 32, 64, 128, 512, 2048, 4096, 1 << 40]


@pytest.mark.slow
def test_rmat_2p20_fp32(h):
    """R-MAT 2^20 vertices, 16 x 2^20 edges, (0.57, 0.19, 0.19, 0.05), FP32
    (0, 1], seed 1 (2.09e10 products, nnz(C) = 9.7e9), C = A*A at full size:
    row_ptr against the oracle's row counts on all 1,048,576 rows; columns
    and values, in full, on 2,000+ rows stratified by numeric bin (every
    bin's boundary rows, lo + 1 and hi outputs, and random rows of each
    bin) and on the contiguous block of the last 65,536 rows."""
    import torch
    A = gen.rmat(20, 16 << 20, seed=1, dtype=np.float32)
    dA = to_dev(A)
    C = h.spgemm(dA, dA)
    torch.cuda.synchronize()
    ref_nnz = oracle.row_nnz(A, A)
    rp = C.row_ptr.cpu().numpy()
    assert rp[0] == 0 and np.array_equal(np.diff(rp), ref_nnz), "row_ptr differs from the oracle's counts"
    assert C.nnz == int(ref_nnz.sum())
    rng = np.random.default_rng(0)
    pick = []
    for lo, hi in zip(NUM_BIN_EDGES[:-1], NUM_BIN_EDGES[1:]):
        inbin = np.nonzero((ref_nnz > lo) & (ref_nnz <= hi))[0]
        assert inbin.size, f"no row in bin ({lo}, {hi}]"
        for edge in (lo + 1, hi):
            pick.append(np.nonzero(ref_nnz == edge)[0][:8])
        pick.append(rng.choice(inbin, min(inbin.size, 300), replace=False))
    pick.append(np.argsort(ref_nnz)[-8:])                 # the largest rows
    pick.append(np.nonzero(ref_nnz == 0)[0][:8])
    rows = np.unique(np.concatenate(pick))
    assert rows.size >= 2000
    block = np.arange(A.nrows - 65536, A.nrows)
    tol = TOL[np.dtype(np.float32)]
    worst = 0.0
    for sel in (rows, block):
        ref = oracle.spgemm(_row_subset(A, sel), A)
        grp, gcol, gval = _device_rows(C, sel)
        worst = max(worst, oracle.compare(grp, gcol, gval, ref, tol))
        del ref, grp, gcol, gval
    # every row strictly increasing (a property at any size), on the device in chunks
    rpd = C.row_ptr
    step = 1 << 28
    for s0 in range(0, C.nnz - 1, step):
        e0 = min(C.nnz - 1, s0 + step)
        d = C.col[s0 + 1:e0 + 1].to(torch.int64) - C.col[s0:e0].to(torch.int64)
        bad = torch.nonzero(d <= 0).flatten() + s0 + 1
        if bad.numel():
            idx = torch.searchsorted(rpd, bad)
            assert torch.all(rpd[idx] == bad), "a row is not strictly increasing"
    print(f"nnz(C) = {C.nnz}, {rows.size} stratified rows + 65,536-row block, max |c-o|/bound = {worst:.3e}")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_merge_full_batches_of_short_rows(h, dtype):
    """16,384 rows with at most 4 outputs each: the merge kernel's row
    ranges hold 64 rows per wave and every 64-row batch fits its staging
    area (the case where all 64 candidate rows are taken at once)."""
    m, n = 16384, 4096
    rng = np.random.default_rng(77)
    A = gen.erdos_renyi(m, n, rng.integers(1, 5, m), seed=78, dtype=dtype)
    # one entry per row of B, in a permuted column
    B = gen.CSR(n, n, np.arange(n + 1, dtype=np.int64), rng.permutation(n).astype(np.int32),
                rng.uniform(-1, 1, n).astype(dtype))
    check_full(h, A, B)


def test_pass_summaries_reach_the_host():
    """The statistics and scan passes publish their summaries straight to
    pinned host memory; the device-copy fallback is not needed."""
    hh = binding.Handle(0)
    try:
        A = gen.laplacian_2d(200)
        dA = to_dev(A)
        for _ in range(5):
            C = hh.spgemm(dA, dA)
        ref = oracle.spgemm(A, A)
        host = C.to_host()
        assert np.array_equal(host.col, ref[1]) and np.array_equal(host.val, ref[2])
        assert hh.summary_fallbacks() == 0
    finally:
        hh.close()


def test_stream_switch_orders_work():
    """A handle moved to another stream right after a call: the next call
    clears the shared workspaces only after the first call's kernels, so
    both products are exact; a call made while torch's current stream is a
    third one allocates C on the handle's stream as well."""
    import torch
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    A = gen.laplacian_2d(512)
    B = gen.erdos_renyi(3000, 3000, 6, seed=71)
    dA, dB = to_dev(A), to_dev(B)
    torch.cuda.synchronize()
    h = binding.Handle(0, stream=s1)
    try:
        with torch.cuda.stream(s1):
            C1 = h.spgemm(dA, dA)
        h.set_stream(s2)
        with torch.cuda.stream(s2):
            C2 = h.spgemm(dB, dB)
        C3 = h.spgemm(dA, dA)               # torch's current stream is the default one here
        torch.cuda.synchronize()
        h.sync()
        for C, M in ((C1, A), (C2, B), (C3, A)):
            host = C.to_host()
            ref = oracle.spgemm(M, M)
            oracle.compare(host.row_ptr, host.col, host.val, ref, TOL[np.dtype(np.float64)])
    finally:
        h.close()


def test_fresh_handles_start_clean():
    """A handle's device info block may reuse memory a destroyed handle
    filled with row counts; a new handle's first call must still report no
    error left over from an earlier call."""
    A = gen.laplacian_2d(150)
    dA = to_dev(A)
    ref = oracle.spgemm(A, A)
    for _ in range(6):
        hh = binding.Handle(0)
        try:
            C = hh.spgemm(dA, dA)
            host = C.to_host()
            assert np.array_equal(host.row_ptr, ref[0]) and np.array_equal(host.col, ref[1])
            hh.sync()
        finally:
            hh.close()


def test_merge_first_products_over_many_scan_tiles(h):
    """Every row's bound falls in the merge bin (at most 5 x 6 products), so
    the fused statistics and merge pass counts all rows and the scan behind
    it needs no look-back; 60,000 rows span eight scan tiles, and the row
    counts range over several values per tile."""
    m = 60000
    rng = np.random.default_rng(91)
    A = gen.erdos_renyi(m, m, rng.integers(0, 6, m), seed=92)
    B = gen.erdos_renyi(m, m, rng.integers(1, 7, m), seed=93)
    check_full(h, A, B)
    rn, tot = h.symbolic(to_dev(A), to_dev(B))
    ref = oracle.row_nnz(A, B)
    assert np.array_equal(rn.cpu().numpy(), ref) and tot == ref.sum()


@pytest.mark.slow
def test_merge_first_scan_over_super_tiles(h):
    """8.4 million rows, all in the merge bin: 2,052 scan tiles, more than
    the 1,024 super-tile sums hold, so a super-tile spans three tiles and a
    tile adds the sums of the super-tiles before its own and then the block
    totals of its own super-tile before it."""
    m = 4096 * 2051 + 1234
    rng = np.random.default_rng(95)
    A = gen.erdos_renyi(m, m, rng.integers(0, 4, m), seed=96)
    B = gen.erdos_renyi(m, m, rng.integers(1, 5, m), seed=97)
    check_full(h, A, B)
    rn, tot = h.symbolic(to_dev(A), to_dev(B))
    ref = oracle.row_nnz(A, B)
    assert np.array_equal(rn.cpu().numpy(), ref) and tot == ref.sum()


def test_validation_accepts_views(h):
    """A problem's view of a packed batch (row_ptr starting above 0 and
    ending below nnz) passes validation and multiplies like the standalone
    matrix; a negative row pointer is rejected."""
    mats = [gen.erdos_renyi(60, 60, 5, seed=61), gen.erdos_renyi(70, 60, 3, seed=62),
            gen.erdos_renyi(60, 60, 4, seed=63)]
    pk = binding.PackedBatch.from_host(mats)
    B = gen.erdos_renyi(60, 50, 4, seed=64)
    view = pk.view(1)
    C = h.spgemm(view, to_dev(B), validate=True)
    ref = oracle.spgemm(mats[1], B)
    host = C.to_host()
    oracle.compare(host.row_ptr, host.col, host.val, ref, TOL[np.dtype(np.float64)])
    bad = binding.DeviceCSR(view.nrows, view.ncols, view.row_ptr.clone(), view.col, view.val)
    bad.row_ptr[0] = -1
    with pytest.raises(binding.MspError) as e:
        h.spgemm(bad, to_dev(B), validate=True)
    assert e.value.name == "MSP_ERR_INVALID_ARG"


@pytest.mark.parametrize("index", range(8))
def test_table4_standins(h, index):
    """C = A*A on the FP32 stand-ins of the paper's eight matrices (Table IV
    shapes and densities), compared with the oracle in full."""
    name, A = gen.TABLE4[index][0], gen.TABLE4[index][3](np.float32)
    err = check_full(h, A, A)
    print(f"{name}: max |c-o|/bound = {err:.3e}")


def test_long_rows_statistics_and_products(h):
    """Rows with more than 256 A entries are taken apart by the statistics
    pass (chunks over whole workgroups; rows of 5,000 to 20,000 entries span
    several chunks); products, features, the plain
    product through that pass (no merge bin) and the one-pass product must
    all match the oracle."""
    A, B = long_rows_case()
    dA, dB = to_dev(A), to_dev(B)
    prod, feat = h.row_features(dA, dB)
    st = oracle.row_stats(A, B)
    assert np.array_equal(prod.cpu().numpy(), st["prod"])
    assert st["prod"][300] == 0 and A.row_ptr[301] - A.row_ptr[300] == 5000
    assert np.allclose(feat.cpu().numpy(), oracle.features(A, B), rtol=2e-6, atol=2e-6)
    check_full(h, A, B, tuning=(1, 0, 4096, 1024, -1))
    check_full(h, A, B)
    from paper_2112_10037_amd import learned
    pred = binding.Predictor(h, learned.fixed_capacity_params(8.0))
    C, stats = h.spgemm_learned(pred, dA, dB)
    got = C.to_host()
    oracle.compare(got.row_ptr, got.col, got.val, oracle.spgemm(A, B), TOL[np.dtype(np.float64)])
    pred.close()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_narrow_bins_concurrent(dtype):
    """Power-law rows (2 to 2,000 entries): many bins hold a few rows each
    and run concurrently on the handle's side streams, each one-row-per-
    workgroup kernel drawing rows from its own queue.  Three calls in a row
    on one handle (the queues must be back at zero after each launch), then
    on a handle queued on a non-default stream: every product equals the
    oracle's, and the row counts of the symbolic pass are exact."""
    import torch
    A = gen.powerlaw_rows(20_000, 1.45, 2, 2_000, seed=81, dtype=dtype)
    ref = oracle.spgemm(A, A)
    dA = to_dev(A)
    tol = TOL[np.dtype(dtype)]
    h = binding.Handle(0)
    try:
        for _ in range(3):
            C = h.spgemm(dA, dA).to_host()
            oracle.compare(C.row_ptr, C.col, C.val, ref, tol)
    finally:
        h.close()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    h = binding.Handle(0, stream=s)
    try:
        with torch.cuda.stream(s):
            C1 = h.spgemm(dA, dA)
            C2 = h.spgemm(dA, dA)
        torch.cuda.synchronize()
        h.sync()
        for C in (C1, C2):
            host = C.to_host()
            oracle.compare(host.row_ptr, host.col, host.val, ref, tol)
    finally:
        h.close()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_group_rows_sorted_across_wave(h, dtype):
    """Rows of 100 to 256 distinct outputs in the 64-lane hash bins, whose
    columns span more than 32 T columns (T the table size): those over 160
    outputs are put in column order by the wave's bitonic sort, the others
    by the rank count; both must match the oracle, ragged tails (outputs
    not a multiple of 64) included."""
    rng = np.random.default_rng(91)
    m, k, n = 3000, 4000, 60_000
    A = gen.erdos_renyi(m, k, rng.integers(7, 17, m), seed=92, dtype=dtype)
    B = gen.erdos_renyi(k, n, 16, seed=93, dtype=dtype)
    ref = oracle.spgemm(A, B)
    outs = np.diff(ref[0])
    assert outs.min() >= 100 and outs.max() <= 256 and (outs > 160).sum() > 1000
    check_full(h, A, B)


def _span_rows(dtype, width, n_out, spans, seed):
    """B with one row per span s in spans: columns 100 and 100 + s - 1 and
    n_out - 2 distinct columns between them; A selects each B row alone,
    then pairs of them (a row's span is then the wider one's)."""
    rng = np.random.default_rng(seed)
    cols = []
    for s in spans:
        mid = rng.choice(np.arange(101, 100 + s - 1), size=n_out - 2, replace=False)
        cols.append(np.sort(np.concatenate([[100, 100 + s - 1], mid])))
    nb = len(spans)
    brp = np.zeros(nb + 1, dtype=np.int64)
    brp[1:] = np.cumsum([len(c) for c in cols])
    B = gen.CSR(nb, width, brp, np.concatenate(cols).astype(np.int32),
                rng.uniform(-1, 1, int(brp[-1])).astype(dtype))
    arows = [[i] for i in range(nb)] + [[i, j] for i in range(nb) for j in range(i + 1, nb)]
    arp = np.zeros(len(arows) + 1, dtype=np.int64)
    arp[1:] = np.cumsum([len(r) for r in arows])
    A = gen.CSR(len(arows), nb, arp, np.concatenate(arows).astype(np.int32),
                rng.uniform(-1, 1, int(arp[-1])).astype(dtype))
    return A, B


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_group_rows_span_bitmap(h, dtype):
    """Rows of the 64-lane hash bins (256 and 512 table slots, T) whose
    columns span less than 32 T columns take their column order from a
    bitmap of the span; wider rows from the sort or the rank count.  The
    symbolic 64-lane bins count such rows (at most 64 A entries, span from
    the B rows' first and last columns under 32 T) with a bitmap too.
    Banded products with half-widths under and past that limit, and rows
    whose span is one column under, at and one over it, each against the
    oracle."""
    for k, w, lim in ((11, 2000, 8192), (11, 2300, 8192), (16, 4000, 16384), (16, 4600, 16384)):
        A = gen.banded_random(30_000, k, w, seed=97 + w, dtype=dtype)
        rp, col, _, _ = oracle.spgemm(A, A)
        outs = np.diff(rp)
        assert outs.max() <= (128 if k == 11 else 256) and np.median(outs) > (64 if k == 11 else 128)
        wide = (col[rp[1:] - 1] - col[rp[:-1]] + 1 >= lim).sum()
        assert (wide == 0) if w in (2000, 4000) else (wide > 5000)
        check_full(h, A, A)
    # 100-output rows take the 256-slot table (span limit 8,192 columns),
    # 200-output rows the 512-slot one (16,384); the rows of pairs of B
    # rows share column 100 and have up to twice the outputs
    for n_out, lim in ((100, 8192), (200, 16384)):
        spans = [lim - 1, lim, lim + 1, lim // 2]
        A, B = _span_rows(dtype, 40_000, n_out, spans, seed=n_out)
        outs = np.diff(oracle.spgemm(A, B)[0])
        assert outs[:len(spans)].min() == n_out
        check_full(h, A, B)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_group_rows_buckets(h, dtype):
    """Whole-wave rows of at least 64 outputs whose columns span 64,000
    (past the span bitmap) are ordered through 64 buckets of 1,000 columns
    while no bucket holds more than 24 keys, else by the rank count (87-88
    outputs) or the wave's sort (211-212 outputs).  Each B row: c0 keys in
    the first bucket, `per` keys mid-way in each of buckets 1-62 and one in
    the last; A selects each B row alone.  c0 = 24 and 25 on both sizes,
    against the oracle."""
    rng = np.random.default_rng(99)
    cols = []
    for per in (1, 3):
        for c0 in (24, 25):
            mid = [1000 * b + 500 + 7 * i for b in range(1, 63) for i in range(per)]
            cols.append(100 + np.array(list(range(c0)) + mid + [63_999]))
    brp = np.zeros(len(cols) + 1, dtype=np.int64)
    brp[1:] = np.cumsum([len(c) for c in cols])
    B = gen.CSR(len(cols), 64_200, brp, np.concatenate(cols).astype(np.int32),
                rng.uniform(-1, 1, int(brp[-1])).astype(dtype))
    A = gen.CSR(len(cols), len(cols), np.arange(len(cols) + 1, dtype=np.int64),
                np.arange(len(cols), dtype=np.int32), rng.uniform(-1, 1, len(cols)).astype(dtype))
    outs = np.diff(oracle.spgemm(A, B)[0])
    assert list(outs) == [87, 88, 211, 212]
    check_full(h, A, B)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n", [400_000, 2_000_000])
def test_block_rows_sorted(h, dtype, n):
    """Rows of about 500 to 4,000 distinct outputs in the workgroup hash bins
    (default tuning).  Those over 512 outputs are put in column order by the
    radix sort when a row's columns span less than 2^20 (400,000 columns),
    else by the bitonic sort whose short-range stages run in the waves'
    registers (2,000,000 columns); every row must match the oracle, ragged
    sizes (not powers of two, not multiples of 128) included."""
    rng = np.random.default_rng(95)
    m, k = 700, 5000
    A = gen.erdos_renyi(m, k, rng.integers(33, 256, m), seed=96, dtype=dtype)
    B = gen.erdos_renyi(k, n, 16, seed=97, dtype=dtype)
    ref = oracle.spgemm(A, B)
    outs = np.diff(ref[0])
    assert outs.min() > 500 and outs.max() <= 4096 and (outs > 2048).sum() > 50
    span = np.array([ref[1][ref[0][i + 1] - 1] - ref[1][ref[0][i]] for i in range(m)])
    assert (span < (1 << 20)).all() if n < (1 << 20) else (span >= (1 << 20)).mean() > 0.9
    check_full(h, A, B)
