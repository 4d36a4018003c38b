"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself through a retyped formula: each
check is an independent fact (hand-worked products, dense matrix algebra in
NumPy, bitset brute force, exact closed forms, algebraic identities) chosen so
that a dropped term, a wrong index, a sign error or a transposed operand in
the oracle fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2112_10037_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _csr(d):
    return gen.CSR(d["nrows"], d["ncols"], np.asarray(d["row_ptr"], np.int64),
                   np.asarray(d["col"], np.int32), np.asarray(d["val"], np.float64))


def _random_sparse(rng, m, k, density, dtype=np.float64):
    pat = rng.random((m, k)) < density
    vals = rng.uniform(-1, 1, (m, k))
    return gen.from_dense(np.where(pat, vals, 0.0).astype(dtype), pattern=pat)


def _full(A, B):
    rp, col, val, bnd = oracle.spgemm(A, B)
    return gen.CSR(A.nrows, B.ncols, rp, col, val), bnd


# --- hand-worked products (FSpGEMM Sec. II-B, Fig. 1) ------------------------

def test_hand_worked_products():
    cases = json.load(open(os.path.join(GOLDEN, "hand_products.json")))["cases"]
    for c in cases:
        A = _csr(c["A"])
        B = A if c["B"] == "A" else _csr(c["B"])
        rp, col, val, _ = oracle.spgemm(A, B)
        assert rp.tolist() == c["C"]["row_ptr"], c["name"]
        assert col.tolist() == c["C"]["col"], c["name"]
        assert val.tolist() == [float(v) for v in c["C"]["val"]], c["name"]


def test_cancellation_keeps_structural_entry():
    # Algorithm 1 merges by adding, never by testing for zero.
    A = gen.from_dense(np.array([[1.0, 1.0]]))
    B = gen.from_dense(np.array([[1.0], [-1.0]]))
    rp, col, val, bnd = oracle.spgemm(A, B)
    assert rp.tolist() == [0, 1] and col.tolist() == [0]
    assert val[0] == 0.0 and bnd[0] == 2.0


# --- dense GEMM on tiny inputs ----------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_dense_gemm_tiny(seed):
    rng = np.random.default_rng(seed)
    m, k, n = (int(x) for x in rng.integers(1, 49, 3))
    da, db = rng.uniform(0.0, 0.6, 2)
    A = _random_sparse(rng, m, k, da)
    B = _random_sparse(rng, k, n, db)
    C, bnd = _full(A, B)
    Ad, Bd = gen.to_dense(A), gen.to_dense(B)
    # structure: the boolean product of the patterns (not value != 0)
    pa = np.zeros((m, k), np.int64)
    pb = np.zeros((k, n), np.int64)
    pa[np.repeat(np.arange(m), np.diff(A.row_ptr)), A.col] = 1
    pb[np.repeat(np.arange(k), np.diff(B.row_ptr)), B.col] = 1
    pat = (pa @ pb) > 0
    r, c = np.nonzero(pat)
    assert C.nnz == pat.sum()
    assert np.array_equal(np.repeat(np.arange(m), np.diff(C.row_ptr)), r)
    assert np.array_equal(C.col, c.astype(np.int32))
    # values against NumPy's dense product, bound scale against |A||B|
    ref = (Ad @ Bd)[r, c]
    refb = (np.abs(Ad) @ np.abs(Bd))[r, c]
    assert np.all(np.abs(C.val - ref) <= 1e-13 * refb)
    assert np.allclose(bnd, refb, rtol=1e-13, atol=0)


# --- identity and permutation: single-term sums, bit-exact -------------------

@pytest.mark.parametrize("seed", range(4))
def test_identity_and_permutation_exact(seed):
    rng = np.random.default_rng(100 + seed)
    m, n = int(rng.integers(1, 60)), int(rng.integers(1, 60))
    A = _random_sparse(rng, m, n, 0.3)
    Im, In = gen.from_dense(np.eye(m)), gen.from_dense(np.eye(n))
    for C, _ in (_full(A, In), _full(Im, A)):
        assert np.array_equal(C.row_ptr, A.row_ptr)
        assert np.array_equal(C.col, A.col)
        assert np.array_equal(C.val, A.val)
    # row permutation P A and column permutation A Q
    p = rng.permutation(m)
    P = gen.from_dense(np.eye(m)[p])
    C, _ = _full(P, A)
    assert np.array_equal(gen.to_dense(C), gen.to_dense(A)[p])
    q = rng.permutation(n)
    Q = gen.from_dense(np.eye(n)[:, q])
    C, _ = _full(A, Q)
    C.check()
    assert np.array_equal(gen.to_dense(C), gen.to_dense(A)[:, q])


# --- transpose identity (AB)^T = B^T A^T, bit-exact ---------------------------

def _transpose(M):
    import scipy.sparse as sp
    s = sp.csr_matrix((M.val, M.col, M.row_ptr), shape=(M.nrows, M.ncols)).T.tocsr()
    s.sort_indices()
    return gen.CSR(M.ncols, M.nrows, s.indptr.astype(np.int64), s.indices.astype(np.int32),
                   s.data.copy())


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_transpose_identity(dtype):
    rng = np.random.default_rng(7)
    A = _random_sparse(rng, 70, 50, 0.15, dtype)
    B = _random_sparse(rng, 50, 90, 0.12, dtype)
    C, _ = _full(A, B)
    Ct, _ = _full(_transpose(B), _transpose(A))
    T = _transpose(C)
    assert np.array_equal(T.row_ptr, Ct.row_ptr)
    assert np.array_equal(T.col, Ct.col)
    assert np.array_equal(T.val, Ct.val)       # same terms, same ascending-k order


# --- brute-force boolean product for nnz(C) ----------------------------------

def test_boolean_bruteforce():
    rng = np.random.default_rng(11)
    for trial in range(6):
        n = int(rng.integers(1, 257))
        A = gen.erdos_renyi(n, n, int(rng.integers(1, min(n, 12) + 1)), seed=trial)
        bits = [0] * n
        for k in range(n):
            for j in A.col[A.row_ptr[k]:A.row_ptr[k + 1]]:
                bits[k] |= 1 << int(j)
        cnt = oracle.row_nnz(A, A)
        rp, col, _, _ = oracle.spgemm(A, A)
        for i in range(n):
            acc = 0
            for k in A.col[A.row_ptr[i]:A.row_ptr[i + 1]]:
                acc |= bits[int(k)]
            assert cnt[i] == bin(acc).count("1")
            row = [j for j in range(n) if acc >> j & 1]
            assert col[rp[i]:rp[i + 1]].tolist() == row


# --- closed forms -------------------------------------------------------------

def test_laplacian2d_square_closed_form():
    n = 1024
    A = gen.laplacian_2d(n)
    assert A.nnz == 5 * n * n - 4 * n
    st = oracle.row_stats(A, A)
    d = np.diff(A.row_ptr)
    assert st["prod"].sum() == int((d.astype(np.int64) ** 2).sum()) == 26_177_544
    rp, col, val, _ = oracle.spgemm(A, A)
    assert rp[-1] == n * n + 4 * n * (n - 1) + 4 * n * (n - 2) + 4 * (n - 1) ** 2 == 13_611_012
    assert np.diff(rp).max() == 13
    # exact values: diagonal 16 + (#neighbours), axis +-1: -8, axis +-2: 1, diagonal: 2
    rows = np.repeat(np.arange(n * n), np.diff(rp))
    off = col.astype(np.int64) - rows
    y, x = rows // n, rows % n
    cy, cx = col // n, col % n
    dy, dx = cy - y, cx - x
    expect = np.zeros_like(val)
    diag = off == 0
    expect[diag] = 16 + (d[rows[diag]] - 1)
    axis1 = (np.abs(dy) + np.abs(dx) == 1)
    expect[axis1] = -8
    axis2 = ((np.abs(dy) == 2) & (dx == 0)) | ((np.abs(dx) == 2) & (dy == 0))
    expect[axis2] = 1
    diag1 = (np.abs(dy) == 1) & (np.abs(dx) == 1)
    expect[diag1] = 2
    assert np.all(diag | axis1 | axis2 | diag1)
    assert np.array_equal(val, expect)


def test_stencil27_interior_rows():
    n = 9
    A = gen.stencil_27(n, seed=3)
    cnt = oracle.row_nnz(A, A)
    z, y, x = np.indices((n, n, n)).reshape(3, -1)
    # each output row reaches +-2 in each direction, clipped to the grid
    span = lambda c: np.minimum(c + 2, n - 1) - np.maximum(c - 2, 0) + 1
    assert np.array_equal(cnt, span(z) * span(y) * span(x))
    assert cnt.max() == 125


def _coarse_expected(n):
    """R A P for the 7-point Laplacian: aggregate sizes s=(sz,sy,sx) in
    {1,2}; diagonal 6*|a| - 2*(#internal edges); a face neighbour couples
    with -(shared face area)."""
    na = (n + 1) // 2
    size = lambda i: 2 if 2 * i + 1 < n else 1
    E = {}
    for az in range(na):
        for ay in range(na):
            for ax in range(na):
                s = (size(az), size(ay), size(ax))
                a = (az * na + ay) * na + ax
                vol = s[0] * s[1] * s[2]
                internal = (s[0] - 1) * s[1] * s[2] + s[0] * (s[1] - 1) * s[2] + s[0] * s[1] * (s[2] - 1)
                E[(a, a)] = 6.0 * vol - 2.0 * internal
                for dim in range(3):
                    for step in (-1, 1):
                        c = [az, ay, ax]
                        c[dim] += step
                        if 0 <= c[dim] < na:
                            b = (c[0] * na + c[1]) * na + c[2]
                            face = vol // s[dim]
                            E[(a, b)] = -float(face)
    return E


@pytest.mark.parametrize("n", [4, 5, 8, 9])
def test_galerkin_closed_form(n):
    A, P, R = gen.galerkin_problem(n)
    AP, _ = _full(A, P)
    ev = 4 * n ** 3 - (6 if n % 2 == 0 else 3) * n ** 2
    assert AP.nnz == ev
    assert np.diff(AP.row_ptr).max() == 4
    Ac, _ = _full(R, AP)
    E = _coarse_expected(n)
    rows = np.repeat(np.arange(Ac.nrows), np.diff(Ac.row_ptr))
    got = {(int(r), int(c)): float(v) for r, c, v in zip(rows, Ac.col, Ac.val)}
    assert got == E
    if n % 2 == 0:
        L = gen.laplacian_3d(n // 2)
        assert np.array_equal(Ac.row_ptr, L.row_ptr) and np.array_equal(Ac.col, L.col)
        assert np.array_equal(Ac.val, 4.0 * L.val)


def test_er_cfg_product_count():
    A = gen.erdos_renyi(4096, 4096, 8, seed=0)
    st = oracle.row_stats(A, A)
    assert st["prod"].sum() == 4096 * 8 * 8
    cnt = oracle.row_nnz(A, A)
    # E|union of 8 random 8-subsets of 4096| = 4096 (1 - (1 - 8/4096)^8) ~ 63.6
    assert abs(cnt.mean() - 4096 * (1 - (1 - 8 / 4096) ** 8)) < 0.2
    assert cnt.max() <= 64


# --- edge cases ----------------------------------------------------------------

def test_empty_and_degenerate():
    for (m, k, n) in [(0, 0, 0), (0, 5, 3), (4, 0, 3), (4, 5, 0), (3, 3, 3)]:
        A = gen.empty(m, k)
        B = gen.empty(k, n)
        rp, col, val, bnd = oracle.spgemm(A, B)
        assert rp.tolist() == [0] * (m + 1) and col.size == 0
    # one column
    A = gen.from_dense(np.ones((5, 1)))
    B = gen.from_dense(np.full((1, 1), 2.0))
    rp, col, val, _ = oracle.spgemm(A, B)
    assert rp.tolist() == [0, 1, 2, 3, 4, 5] and val.tolist() == [2.0] * 5


def test_row_blocks_match_whole():
    A = gen.rmat(10, 8 << 10, seed=2, dtype=np.float64)
    rp, col, val, bnd = oracle.spgemm(A, A)
    for r0, r1 in [(0, 100), (100, 517), (517, 1024)]:
        brp, bcol, bval, bbnd = oracle.spgemm(A, A, r0, r1)
        s, e = rp[r0], rp[r1]
        assert np.array_equal(brp, rp[r0:r1 + 1] - s)
        assert np.array_equal(bcol, col[s:e]) and np.array_equal(bval, val[s:e])


def test_f32_inputs_promote_exactly():
    A64 = gen.rmat(9, 8 << 9, seed=4, dtype=np.float64)
    A32 = A64.astype(np.float32)
    A64e = A32.astype(np.float64)          # the f32 values, held exactly in f64
    r32 = oracle.spgemm(A32, A32)
    r64 = oracle.spgemm(A64e, A64e)
    for a, b in zip(r32, r64):
        assert np.array_equal(a, b)


def test_compare_rejects_planted_mistakes():
    A = gen.erdos_renyi(64, 64, 6, seed=9)
    ref = oracle.spgemm(A, A)
    rp, col, val, _ = ref
    oracle.compare(rp, col, val, ref, 1e-12)
    bad = val.copy()
    bad[5] += 1e-6
    with pytest.raises(AssertionError):
        oracle.compare(rp, col, bad, ref, 1e-12)
    badc = col.copy()
    badc[3] += 1
    with pytest.raises(AssertionError):
        oracle.compare(rp, badc, val, ref, 1e-12)


def test_row_stats_definitions():
    A = gen.from_dense(np.array([[1, 0, 1, 0], [0, 0, 0, 0], [0, 1, 0, 1], [1, 1, 1, 1.0]]))
    B = gen.from_dense(np.array([[0, 1, 1, 0], [0, 0, 0, 0], [1, 0, 0, 1], [0, 0, 1, 0.0]]))
    s = oracle.row_stats(A, B)
    assert s["nnz_a"].tolist() == [2, 0, 2, 4]
    assert s["prod"].tolist() == [4, 0, 1, 5]
    assert s["min_b"].tolist() == [2, 0, 0, 0]
    assert s["max_b"].tolist() == [2, 0, 1, 2]
    assert s["span"].tolist() == [3, 0, 0, 3]
