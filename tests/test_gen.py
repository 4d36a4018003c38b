"""Generators: determinism, canonical CSR, the structure each family promises."""
import hashlib

import numpy as np

from paper_2112_10037_amd import gen


def _digest(m):
    h = hashlib.sha256()
    for a in (m.row_ptr, m.col, m.val):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_deterministic():
    assert _digest(gen.erdos_renyi(4096, 4096, 8, seed=0)) == _digest(gen.erdos_renyi(4096, 4096, 8, seed=0))
    assert _digest(gen.rmat(12, 16 << 12, seed=1)) == _digest(gen.rmat(12, 16 << 12, seed=1))
    assert _digest(gen.rmat(12, 16 << 12, seed=1)) != _digest(gen.rmat(12, 16 << 12, seed=2))


def test_er_exact_k():
    A = gen.erdos_renyi(4096, 4096, 8, seed=0)
    A.check()
    assert np.all(np.diff(A.row_ptr) == 8)
    assert A.val.min() >= -1 and A.val.max() <= 1
    k = np.random.default_rng(3).integers(4, 33, 1000)
    B = gen.erdos_renyi(1000, 5000, k, seed=5)
    B.check()
    assert np.array_equal(np.diff(B.row_ptr), k)


def test_stencils():
    L = gen.laplacian_2d(16)
    L.check()
    assert L.nnz == 5 * 256 - 4 * 16
    assert set(np.unique(L.val).tolist()) == {-1.0, 4.0}
    L3 = gen.laplacian_3d(6)
    L3.check()
    assert L3.nnz == 7 * 216 - 6 * 36
    S = gen.stencil_27(7, seed=1)
    S.check()
    assert np.diff(S.row_ptr).max() == 27


def test_rmat():
    A = gen.rmat(14, 16 << 14, seed=1)
    A.check()
    assert A.val.dtype == np.float32 and A.val.min() > 0 and A.val.max() <= 1
    assert A.nnz < 16 << 14
    d = np.diff(A.row_ptr)
    assert d.max() > 20 * d.mean()          # power-law skew


def test_prolongator():
    P, R = gen.aggregation_prolongator(5)
    P.check()
    R.check()
    assert P.nnz == R.nnz == 125 and R.nrows == 27
    dense_p = gen.to_dense(P)
    assert np.array_equal(gen.to_dense(R), dense_p.T)


def test_suite():
    s = gen.learned_suite()
    assert len(s) == 64 and sum(m.held_out for m in s) == 16
    assert {m.family for m in s} == {"stencil27", "er", "rmat"}
    m = s[1].build(scale_down=8)
    m.check()


def test_table4_standins_match_the_table_shapes():
    """The stand-ins for the paper's eight matrices (Sec. V-A, Table IV) have
    its dimensions within 5% and its densities within 15%, FP32, canonical."""
    for (name, rows, dens, _), (name2, M) in zip(gen.TABLE4, gen.table4_standins()):
        assert name == name2
        M.check()
        assert M.val.dtype == np.float32 and M.nrows == M.ncols
        assert abs(M.nrows / rows - 1) < 0.05, name
        assert abs(M.nnz / M.nrows / M.ncols / dens - 1) < 0.15, name


def test_banded_random_rows():
    M = gen.banded_random(500, 9, 20, seed=3)
    M.check()
    r = np.repeat(np.arange(500), np.diff(M.row_ptr))
    assert np.all(np.abs(M.col.astype(np.int64) - r) <= 20)
    assert np.all(np.diff(M.row_ptr) == 9)
    assert np.all(np.bincount(r[M.col == r], minlength=500) == 1)    # every row holds its diagonal


def test_powerlaw_rows_lengths():
    M = gen.powerlaw_rows(20000, 1.45, 2, 500, seed=9)
    M.check()
    k = np.diff(M.row_ptr)
    assert k.min() >= 2 and k.max() <= 500
    assert 4.5 < k.mean() < 7.0 and np.median(k) <= 4
