"""CPU oracle for C = A*B (row-wise Gustavson, FSpGEMM Sec. II-B).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this package.  The product library never
links, calls or loads it, and it imports nothing from the product package:
matrices are passed in as any object with ``nrows, ncols, row_ptr (int64),
col (int32), val (f32/f64)`` attributes.

The arithmetic lives in ``spgemm_oracle.c`` (plain C, FP64 dense accumulator,
``-ffp-contract=off``) and ``mlp.py`` (NumPy FP64).  ``build()`` compiles the
C part with gcc; the shared object sits next to the source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spgemm_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(src: str = _SRC, out: str = _SO) -> str:
    """Compile the C oracle (always recompiles).  ``src``/``out`` are
    overridden only by the mutation tests, which compile planted mistakes."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-Wall", src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def use_library(path: str | None):
    """Point the wrappers at another build of the oracle source (mutation
    tests only); ``None`` restores the default.  Returns the previous handle."""
    global _lib
    prev = _lib
    _lib = None if path is None else _bind(ctypes.CDLL(path))
    return prev


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_SO))
    return _lib


def _bind(lib):
    p = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.oracle_row_nnz.argtypes = [i64, i64, i64, p, p, p, p, p]
    lib.oracle_row_nnz.restype = ctypes.c_int
    lib.oracle_spgemm_rows.argtypes = [i64, i64, i64, p, p, p, p, p, p,
                                       ctypes.c_int, p, p, p, p]
    lib.oracle_spgemm_rows.restype = ctypes.c_int
    lib.oracle_row_stats.argtypes = [i64, i64, p, p, p, p, p, p, p, p, p]
    lib.oracle_row_stats.restype = None
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def _canon(m):
    rp = np.ascontiguousarray(m.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(m.col, dtype=np.int32)
    val = np.ascontiguousarray(m.val)
    if val.dtype not in (np.float32, np.float64):
        val = val.astype(np.float64)
    return rp, col, val


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def row_nnz(A, B, r0: int = 0, r1: int | None = None) -> np.ndarray:
    """|union of column sets| per output row, rows [r0, r1)."""
    if A.ncols != B.nrows:
        raise ValueError("shape mismatch")
    r1 = A.nrows if r1 is None else r1
    lib = _load()
    a_rp, a_col, _ = _canon(A)
    b_rp, b_col, _ = _canon(B)
    out = np.zeros(r1 - r0, dtype=np.int64)
    if r1 > r0:
        rc = lib.oracle_row_nnz(r0, r1, B.ncols, _ptr(a_rp), _ptr(a_col), _ptr(b_rp),
                                _ptr(b_col), _ptr(out))
        if rc:
            raise MemoryError("oracle_row_nnz failed")
    return out


def spgemm(A, B, r0: int = 0, r1: int | None = None):
    """Rows [r0, r1) of C = A*B.

    Returns ``(row_ptr, col, val, bnd)``: row_ptr int64 of length r1-r0+1
    starting at 0, sorted int32 columns, FP64 values and the FP64 bound scale
    sum_k |a_ik||b_kj| of every entry.
    """
    if A.ncols != B.nrows:
        raise ValueError("shape mismatch")
    r1 = A.nrows if r1 is None else r1
    lib = _load()
    a_rp, a_col, a_val = _canon(A)
    b_rp, b_col, b_val = _canon(B)
    if a_val.dtype != b_val.dtype:
        raise TypeError("A and B value types differ")
    cnt = row_nnz(A, B, r0, r1)
    rp = np.zeros(r1 - r0 + 1, dtype=np.int64)
    np.cumsum(cnt, out=rp[1:])
    nnz = int(rp[-1])
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(nnz, dtype=np.float64)
    bnd = np.zeros(nnz, dtype=np.float64)
    if r1 > r0:
        rc = lib.oracle_spgemm_rows(r0, r1, B.ncols, _ptr(a_rp), _ptr(a_col), _ptr(a_val),
                                    _ptr(b_rp), _ptr(b_col), _ptr(b_val),
                                    int(a_val.dtype == np.float32), _ptr(rp),
                                    _ptr(col), _ptr(val), _ptr(bnd))
        if rc:
            raise RuntimeError(f"oracle_spgemm_rows failed ({rc})")
    return rp, col, val, bnd


def row_stats(A, B, r0: int = 0, r1: int | None = None) -> dict:
    """nnz_a, prod, min_b, max_b, span per row of A against B (int64 arrays)."""
    r1 = A.nrows if r1 is None else r1
    lib = _load()
    a_rp, a_col, _ = _canon(A)
    b_rp, b_col, _ = _canon(B)
    n = r1 - r0
    out = {k: np.zeros(n, dtype=np.int64) for k in ("nnz_a", "prod", "min_b", "max_b", "span")}
    if n > 0:
        lib.oracle_row_stats(r0, r1, _ptr(a_rp), _ptr(a_col), _ptr(b_rp), _ptr(b_col),
                             _ptr(out["nnz_a"]), _ptr(out["prod"]), _ptr(out["min_b"]),
                             _ptr(out["max_b"]), _ptr(out["span"]))
    return out


def features(A, B) -> np.ndarray:
    """The 8 per-row predictor inputs (FP64), from ``row_stats``:
    log2(1+x)/16 of nnz_a, prod, min_b, mean_b, max_b and ncols(B); then
    min(1, prod/ncols(B)) and span/ncols(B)."""
    s = row_stats(A, B)
    n = max(int(B.ncols), 1)
    nnz_a = s["nnz_a"].astype(np.float64)
    prod = s["prod"].astype(np.float64)
    mean_b = np.divide(prod, nnz_a, out=np.zeros_like(prod), where=nnz_a > 0)
    f = np.empty((A.nrows, 8), dtype=np.float64)
    f[:, 0] = np.log2(1.0 + nnz_a) / 16.0
    f[:, 1] = np.log2(1.0 + prod) / 16.0
    f[:, 2] = np.log2(1.0 + s["min_b"]) / 16.0
    f[:, 3] = np.log2(1.0 + mean_b) / 16.0
    f[:, 4] = np.log2(1.0 + s["max_b"]) / 16.0
    f[:, 5] = np.log2(1.0 + float(B.ncols)) / 16.0
    f[:, 6] = np.minimum(1.0, prod / n)
    f[:, 7] = s["span"] / n
    return f


def omar_distinct(A, group: int) -> int:
    """B-row reads of the buffering scheme of Sec. IV-A (Eq. (1)): with A's
    rows taken in groups of ``group`` consecutive rows (the last group may be
    shorter), one read of B row k per group whose rows hold column k.  The
    number of distinct (group, column) pairs, by the definition: the union of
    the columns of each group's rows, summed over groups."""
    rp = np.asarray(A.row_ptr, dtype=np.int64)
    rows = np.repeat(np.arange(A.nrows, dtype=np.int64), np.diff(rp))
    keys = (rows // int(group)) * max(int(A.ncols), 1) + np.asarray(A.col, dtype=np.int64)
    return int(np.unique(keys).size)


def omar(A, group: int) -> float:
    """OMAR of Eq. (1) in percent: the B-row reads saved, over nnz(A)."""
    nnz = int(A.row_ptr[-1]) if A.nrows else 0
    return 100.0 * (nnz - omar_distinct(A, group)) / nnz if nnz else 0.0


def compare(rp, col, val, ref, tol: float):
    """Check a computed C block against an oracle block ``ref`` (the tuple
    returned by :func:`spgemm`).  Structure must be identical; every value
    must satisfy |c - o| <= tol * bnd (with bnd = 0 requiring c == 0).
    Returns the largest |c - o| / bnd over entries with bnd > 0."""
    o_rp, o_col, o_val, o_bnd = ref
    rp = np.asarray(rp, dtype=np.int64)
    rp = rp - rp[0]
    if not np.array_equal(rp, o_rp):
        bad = np.nonzero(rp != o_rp)[0]
        raise AssertionError(f"row_ptr differs first at local row {bad[0] - 1 if bad[0] else 0}")
    if not np.array_equal(np.asarray(col, np.int32), o_col):
        bad = np.nonzero(np.asarray(col) != o_col)[0][0]
        raise AssertionError(f"col differs first at entry {bad}: {col[bad]} vs {o_col[bad]}")
    c = np.asarray(val, dtype=np.float64)
    err = np.abs(c - o_val)
    zero = o_bnd == 0
    if np.any(c[zero] != 0):
        raise AssertionError("nonzero value where every term is zero")
    ok = err <= tol * o_bnd
    if not np.all(ok):
        i = np.nonzero(~ok)[0][0]
        raise AssertionError(f"value out of bound at entry {i}: {c[i]!r} vs {o_val[i]!r}, "
                             f"bound {tol * o_bnd[i]!r}")
    nz = ~zero
    return float(np.max(err[nz] / o_bnd[nz])) if np.any(nz) else 0.0
