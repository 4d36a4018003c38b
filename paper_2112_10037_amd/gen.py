"""Seeded synthetic input generators (CSR, host memory).

This module produces inputs only: sparsity patterns and values.  It holds none
of the SpGEMM arithmetic and is shared by the oracle-side tests and the HIP
path's tests and benchmark, which is the only code the two sides share.

Every random draw comes from ``numpy.random.default_rng(seed)`` (PCG64, the
published O'Neill generator with NumPy's SeedSequence seeding).  Values
uniform in [-1, 1] are ``2u - 1``; values uniform in (0, 1] are ``1 - u``;
in both ``u`` is a 53-bit uniform in [0, 1).  Values are drawn in CSR order
after the pattern is fixed.

Workload shapes follow the matrices the FSpGEMM evaluation uses
(Sec. V-A, Table IV: SuiteSparse stencil-like, circuit and web graphs),
which are not available here; these synthetic families stand in for them:
Erdos-Renyi rows with an exact count, 2D/3D finite-difference stencils and
R-MAT power-law graphs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    """A CSR matrix in host memory: int64 row_ptr, int32 col, f32/f64 val."""

    nrows: int
    ncols: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1]) if self.row_ptr.size else 0

    @property
    def dtype(self):
        return self.val.dtype

    def astype(self, dtype) -> "CSR":
        return CSR(self.nrows, self.ncols, self.row_ptr, self.col,
                   self.val.astype(dtype))

    def check(self) -> None:
        """Assert the canonical-CSR contract (monotone, sorted, unique, in range)."""
        assert self.row_ptr.dtype == np.int64 and self.col.dtype == np.int32
        assert self.row_ptr.shape == (self.nrows + 1,)
        assert self.row_ptr[0] == 0 and self.col.size == self.nnz == self.val.size
        assert np.all(np.diff(self.row_ptr) >= 0)
        if self.nnz:
            assert self.col.min() >= 0 and self.col.max() < self.ncols
            d = np.diff(self.col.astype(np.int64))
            starts = self.row_ptr[1:-1]
            inner = np.ones(self.nnz - 1, dtype=bool)
            inner[starts[(starts > 0) & (starts < self.nnz)] - 1] = False
            assert np.all(d[inner] > 0), "columns must be strictly increasing in a row"


def _from_coo(nrows, ncols, rows, cols, vals=None, dtype=np.float64):
    """Sort (row, col) pairs and build CSR; pairs must already be unique."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    counts = np.bincount(rows, minlength=nrows)
    row_ptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    v = None if vals is None else np.asarray(vals)[order].astype(dtype)
    return row_ptr, cols.astype(np.int32), v


def _uniform_pm1(rng, n, dtype):
    return (2.0 * rng.random(n) - 1.0).astype(dtype)


def from_dense(d: np.ndarray, pattern: np.ndarray | None = None) -> CSR:
    """CSR of a dense array; ``pattern`` (bool) marks stored entries (explicit
    zeros allowed).  Default pattern: the nonzeros of ``d``."""
    d = np.asarray(d)
    pat = (d != 0) if pattern is None else np.asarray(pattern, dtype=bool)
    r, c = np.nonzero(pat)
    row_ptr = np.zeros(d.shape[0] + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=d.shape[0]), out=row_ptr[1:])
    return CSR(d.shape[0], d.shape[1], row_ptr, c.astype(np.int32), d[r, c].copy())


def to_dense(a: CSR) -> np.ndarray:
    out = np.zeros((a.nrows, a.ncols), dtype=np.float64)
    rows = np.repeat(np.arange(a.nrows), np.diff(a.row_ptr))
    out[rows, a.col.astype(np.int64)] = a.val
    return out


def empty(nrows: int, ncols: int, dtype=np.float64) -> CSR:
    return CSR(nrows, ncols, np.zeros(nrows + 1, np.int64),
               np.zeros(0, np.int32), np.zeros(0, dtype))


# ---------------------------------------------------------------------------
# Erdos-Renyi rows with an exact nonzero count
# ---------------------------------------------------------------------------

def erdos_renyi(nrows: int, ncols: int, k, seed: int, dtype=np.float64) -> CSR:
    """Each row gets exactly k[i] distinct columns, uniform without replacement.

    ``k`` is an int or a length-nrows array.  Each row draws kmax uniform
    columns; a row in which a column repeats is redrawn without replacement
    (``Generator.choice``).  Row i keeps the first k[i] in draw order (a
    uniform k[i]-subset), then sorts them.  Values U[-1, 1].
    """
    rng = np.random.default_rng(seed)
    kk = np.full(nrows, int(k), dtype=np.int64) if np.isscalar(k) else np.asarray(k, np.int64)
    kmax = int(kk.max()) if nrows else 0
    if kmax > ncols:
        raise ValueError("k exceeds ncols")
    if nrows == 0 or kmax == 0:
        return empty(nrows, ncols, dtype)
    draw = rng.integers(0, ncols, size=(nrows, kmax), dtype=np.int64)
    if kmax > 1:
        s = np.sort(draw, axis=1)
        bad = np.nonzero(np.any(s[:, 1:] == s[:, :-1], axis=1))[0]
        for r in bad:               # rows with a repeat: an exact draw without replacement
            draw[r] = rng.choice(ncols, size=kmax, replace=False)
    keep = np.arange(kmax)[None, :] < kk[:, None]
    draw = np.where(keep, draw, np.iinfo(np.int64).max)
    draw.sort(axis=1)          # kept columns sorted first, sentinels last
    cols = draw[keep]
    row_ptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(kk, out=row_ptr[1:])
    val = _uniform_pm1(rng, int(row_ptr[-1]), dtype)
    return CSR(nrows, ncols, row_ptr, cols.astype(np.int32), val)


def banded_random(n: int, k: int, halfwidth: int, seed: int, dtype=np.float64) -> CSR:
    """n x n: row i holds the diagonal and k - 1 other distinct columns drawn
    uniformly from the band [i - w, i + w] clipped to [0, n) (fewer when the
    clipped band is narrower), the locality of a mesh-based matrix.
    Values U[-1, 1] in CSR order."""
    rng = np.random.default_rng(seed)
    rows, cols = [np.arange(n, dtype=np.int64)], [np.arange(n, dtype=np.int64)]
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(0, i - halfwidth)
    size = np.minimum(n - 1, i + halfwidth) - lo          # band width minus the diagonal
    kk = np.minimum(k - 1, size)
    m = int(kk.max()) if n else 0
    if m > 0:
        draw = (rng.random((n, m)) * size[:, None]).astype(np.int64)
        s = np.sort(draw, axis=1)
        bad = np.nonzero(np.any((s[:, 1:] == s[:, :-1]) & (np.arange(1, m)[None, :] < kk[:, None]), axis=1))[0]
        for r in bad:
            draw[r, :kk[r]] = rng.choice(size[r], size=int(kk[r]), replace=False)
        c = lo[:, None] + draw
        c = np.where(c >= i[:, None], c + 1, c)            # skip the diagonal
        keep = np.arange(m)[None, :] < kk[:, None]
        rows.append(np.repeat(i, kk))
        cols.append(c[keep])
    rr, cc = np.concatenate(rows), np.concatenate(cols)
    row_ptr, col, _ = _from_coo(n, n, rr, cc)
    return CSR(n, n, row_ptr, col, _uniform_pm1(rng, col.size, dtype))


def powerlaw_rows(n: int, alpha: float, kmin: int, kmax: int, seed: int, dtype=np.float64) -> CSR:
    """n x n with power-law row lengths: k_i = floor(kmin (1 - u)^(-1/alpha))
    clipped to [kmin, kmax] (mean about kmin alpha / (alpha - 1)), columns
    uniform without replacement as in erdos_renyi.  Values U[-1, 1]."""
    rng = np.random.default_rng(seed)
    k = np.floor(kmin * (1.0 - rng.random(n)) ** (-1.0 / alpha)).astype(np.int64)
    k = np.clip(k, kmin, min(kmax, n))
    # every row's columns in one draw; rows where a column repeats are
    # redrawn without replacement
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(k, out=row_ptr[1:])
    rid = np.repeat(np.arange(n, dtype=np.int64), k)
    cols = rng.integers(0, n, size=int(row_ptr[-1]), dtype=np.int64)
    cols = cols[np.lexsort((cols, rid))]
    dup = np.nonzero((cols[1:] == cols[:-1]) & (rid[1:] == rid[:-1]))[0]
    for r in np.unique(rid[dup + 1]):
        cols[row_ptr[r]:row_ptr[r + 1]] = np.sort(rng.choice(n, size=int(k[r]), replace=False))
    return CSR(n, n, row_ptr, cols.astype(np.int32), _uniform_pm1(rng, cols.size, dtype))


# Stand-ins for the eight matrices of the paper's evaluation (Sec. V-A,
# Table IV: SuiteSparse matrices, not available here), with the dimensions
# and densities the table gives and a structure of the same kind: 3D
# 27-point stencils for the FEM Poisson and filter matrices, banded random
# rows for the FEM sphere and offshore meshes, uniform rows for the DNA
# electrophoresis and economics matrices, power-law rows for the circuit and
# an R-MAT graph for the web crawl.  FP32, as in the paper.
TABLE4 = [
    # name, rows, density (Table IV), recipe
    ("poisson3Da", 14_000, 1.9e-3, lambda dt: stencil_27(24, seed=4001, dtype=dt)),
    ("2cubes_sphere", 101_000, 1.6e-4, lambda dt: banded_random(101_000, 16, 2_170, seed=4002, dtype=dt)),
    ("filter3D", 106_000, 2.4e-4, lambda dt: stencil_27(47, seed=4003, dtype=dt)),
    ("cage12", 130_000, 1.2e-4, lambda dt: erdos_renyi(130_000, 130_000, 16, seed=4004, dtype=dt)),
    ("scircuit", 171_000, 3.3e-5, lambda dt: powerlaw_rows(171_000, 1.45, 2, 2_000, seed=4005, dtype=dt)),
    ("mac_econ_fwd500", 207_000, 3.0e-5, lambda dt: erdos_renyi(207_000, 207_000, 6, seed=4006, dtype=dt)),
    ("offshore", 260_000, 6.3e-5, lambda dt: banded_random(260_000, 16, 4_070, seed=4007, dtype=dt)),
    ("webbase-1M", 1_000_000, 3.1e-6, lambda dt: rmat(20, int(3.2 * 2 ** 20), seed=4008, dtype=dt)),
]


def table4_standins(dtype=np.float32):
    """[(name, CSR)] of the Table IV stand-ins (FP32 unless told)."""
    return [(name, recipe(dtype)) for name, _, _, recipe in TABLE4]


# ---------------------------------------------------------------------------
# Finite-difference stencils (Dirichlet boundary: off-grid neighbours dropped)
# ---------------------------------------------------------------------------

def _stencil(dims, offsets, vals_by_offset, rng=None, dtype=np.float64) -> CSR:
    dims = tuple(int(d) for d in dims)
    N = int(np.prod(dims)) if dims else 0
    coords = np.indices(dims).reshape(len(dims), -1)  # row r -> (z, y, x) lexicographic
    strides = np.array([int(np.prod(dims[i + 1:])) for i in range(len(dims))], dtype=np.int64)
    rows_l, cols_l, vals_l = [], [], []
    for off, v in zip(offsets, vals_by_offset):
        nb = coords + np.array(off, dtype=np.int64)[:, None]
        ok = np.all((nb >= 0) & (nb < np.array(dims)[:, None]), axis=0)
        r = np.nonzero(ok)[0]
        c = (nb[:, ok] * strides[:, None]).sum(axis=0)
        rows_l.append(r)
        cols_l.append(c)
        vals_l.append(np.full(r.size, v, dtype=np.float64))
    row_ptr, col, val = _from_coo(N, N, np.concatenate(rows_l), np.concatenate(cols_l),
                                  np.concatenate(vals_l), dtype)
    if rng is not None:
        val = _uniform_pm1(rng, val.size, dtype)
    return CSR(N, N, row_ptr, col, val)


def laplacian_2d(n: int, dtype=np.float64) -> CSR:
    """2D 5-point Laplacian on an n x n grid: diagonal 4, neighbours -1."""
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    vals = [4.0, -1.0, -1.0, -1.0, -1.0]
    return _stencil((n, n), offs, vals, dtype=dtype)


def laplacian_3d(n: int, dtype=np.float64) -> CSR:
    """3D 7-point Laplacian on an n^3 grid: diagonal 6, neighbours -1."""
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    vals = [6.0] + [-1.0] * 6
    return _stencil((n, n, n), offs, vals, dtype=dtype)


def stencil_27(n: int, seed: int, dtype=np.float64) -> CSR:
    """3D 27-point stencil pattern on an n^3 grid, values U[-1, 1]."""
    offs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    return _stencil((n, n, n), offs, [0.0] * 27, rng=np.random.default_rng(seed), dtype=dtype)


# ---------------------------------------------------------------------------
# R-MAT power-law graphs
# ---------------------------------------------------------------------------

def rmat(scale: int, nedges: int, a=0.57, b=0.19, c=0.19, seed: int = 1,
         dtype=np.float32, chunk: int = 1 << 22) -> CSR:
    """R-MAT graph on 2^scale vertices (Chakrabarti, Zhan, Faloutsos 2004).

    Each of ``nedges`` directed edges descends ``scale`` levels; at each level
    one uniform u picks quadrant (0,0) if u < a, (0,1) if u < a+b, (1,0) if
    u < a+b+c, else (1,1), the most significant bit first.  No per-level
    noise, no symmetrisation; self-loops kept; duplicate edges merged after
    all edges are drawn.  One value per unique entry, in CSR order, uniform
    in (0, 1].
    """
    rng = np.random.default_rng(seed)
    n = 1 << scale
    keys = np.empty(nedges, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for s in range(0, nedges, chunk):
        e = min(nedges, s + chunk)
        r = np.zeros(e - s, dtype=np.int64)
        q = np.zeros(e - s, dtype=np.int64)
        for lvl in range(scale):
            u = rng.random(e - s)
            bit = np.int64(1) << np.int64(scale - 1 - lvl)
            rbit = u >= ab
            cbit = ((u >= a) & (u < ab)) | (u >= abc)
            r |= np.where(rbit, bit, 0)
            q |= np.where(cbit, bit, 0)
        keys[s:e] = (r << np.int64(scale)) | q
    keys = np.unique(keys)
    rows = keys >> np.int64(scale)
    cols = (keys & np.int64(n - 1)).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    val = (1.0 - rng.random(keys.size)).astype(dtype)
    return CSR(n, n, row_ptr, cols, val)


# ---------------------------------------------------------------------------
# Aggregation prolongator for the Galerkin triple product
# ---------------------------------------------------------------------------

def aggregation_prolongator(n: int, dtype=np.float64):
    """Piecewise-constant prolongator P (n^3 x na^3, na = ceil(n/2)) over 2x2x2
    aggregates, values 1.0, and its transpose R generated directly as CSR.

    Fine point (z, y, x) belongs to aggregate (z//2, y//2, x//2); with odd n
    the last aggregate in each direction is partial.
    """
    na = (n + 1) // 2
    z, y, x = np.indices((n, n, n)).reshape(3, -1)
    agg = ((z // 2) * na + (y // 2)) * na + (x // 2)
    N, Na = n ** 3, na ** 3
    P = CSR(N, Na, np.arange(N + 1, dtype=np.int64), agg.astype(np.int32),
            np.ones(N, dtype=dtype))
    order = np.argsort(agg, kind="stable")
    r_ptr = np.zeros(Na + 1, dtype=np.int64)
    np.cumsum(np.bincount(agg, minlength=Na), out=r_ptr[1:])
    R = CSR(Na, N, r_ptr, order.astype(np.int32), np.ones(N, dtype=dtype))
    return P, R


def galerkin_problem(n: int, dtype=np.float64):
    """(A, P, R) for one Galerkin product R*(A*P) with a 7-point Laplacian."""
    A = laplacian_3d(n, dtype)
    P, R = aggregation_prolongator(n, dtype)
    return A, P, R


def galerkin_sizes(nprob: int = 512, lo: int = 16, hi: int = 64, seed: int = 5) -> np.ndarray:
    """Grid sides n ~ U{lo..hi} for the batched Galerkin workload."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=nprob)


# ---------------------------------------------------------------------------
# Mixed suite for the learned output-size predictor
# ---------------------------------------------------------------------------

@dataclass
class SuiteMember:
    index: int
    seed: int
    family: str        # "stencil27" | "er" | "rmat"
    param: int         # stencil side n, or log2(rows) for ER / R-MAT
    degree: int        # R-MAT edge factor (0 otherwise)
    held_out: bool

    def build(self, scale_down: int = 0, dtype=np.float64) -> CSR:
        """Materialise the matrix; ``scale_down`` shrinks it by 2^scale_down
        rows (used by quick tests; the full suite uses 0)."""
        rng = np.random.default_rng(self.seed)
        if self.family == "stencil27":
            n = max(4, int(round(self.param / (2 ** (scale_down / 3)))))
            return stencil_27(n, self.seed, dtype)
        if self.family == "er":
            m = 1 << max(6, self.param - scale_down)
            k = rng.integers(4, 33, size=m)
            return erdos_renyi(m, m, k, self.seed + 7919, dtype)
        s = max(6, self.param - scale_down)
        return rmat(s, self.degree << s, seed=self.seed, dtype=dtype).astype(dtype)


def learned_suite(count: int = 64, seed_base: int = 1000):
    """64 seeded members: family by seed mod 3 (27-point stencil, ER with
    4..32 nonzeros per row, R-MAT with degree 8..32); sizes 2^16..2^20 rows
    (R-MAT capped at 2^18 so that C fits in device memory); members whose
    index is 3 mod 4 are held out (16 of 64)."""
    out = []
    for i in range(count):
        seed = seed_base + i
        rng = np.random.default_rng(seed)
        fam = ("stencil27", "er", "rmat")[seed % 3]
        if fam == "stencil27":
            param, deg = int(rng.integers(41, 102)), 0
        elif fam == "er":
            param, deg = int(rng.integers(16, 21)), 0
        else:
            param, deg = int(rng.integers(16, 19)), int(rng.integers(8, 33))
        out.append(SuiteMember(i, seed, fam, param, deg, i % 4 == 3))
    return out


# ---------------------------------------------------------------------------
# Random draws of the predictor's training (passed to both sides as inputs)
# ---------------------------------------------------------------------------

# (shape, fan_in) of W1 b1 W2 b2 W3 b3; fan_in None marks a bias
MLP_LAYOUT = [((64, 8), 8), ((64,), None), ((64, 64), 64), ((64,), None),
              ((64,), 64), ((1,), None)]


def mlp_init(seed: int) -> np.ndarray:
    """He-uniform initial weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)) with zero
    biases, flat in the order W1[64][8] b1 W2[64][64] b2 W3[64] b3 (FP64)."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape, fan_in in MLP_LAYOUT:
        n = int(np.prod(shape))
        if fan_in is None:
            parts.append(np.zeros(n))
        else:
            parts.append(rng.uniform(-1.0, 1.0, n) * np.sqrt(6.0 / fan_in))
    return np.concatenate(parts)


def minibatch_indices(nrows: int, batch: int, steps: int, seed: int) -> np.ndarray:
    """steps x batch row indices drawn uniformly with replacement (int32)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, nrows, size=(steps, batch), dtype=np.int64).astype(np.int32)
