"""Host-side pieces of bench.py (no GPU): the refusal of more than one GPU,
the hash that keeps a measured traffic figure tied to the kernel sources'
code, and the algorithmic byte counts the roofline is read against, each
against a hand-worked case."""
import importlib.util
import os
import subprocess
import sys

import numpy as np

from paper_2112_10037_amd import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""                      # no JSON line


def test_code_only_ignores_comments_and_blank_lines():
    b = _bench()
    a = "int f(int x) {  // the input\n    return x + 1; /* one\n more */\n\n}\n"
    c = "int f(int x) {\n    return x + 1;\n}\n"
    assert b._code_only(a) == b._code_only(c)
    assert b._code_only(a) != b._code_only(c.replace("x + 1", "x + 2"))


def test_sources_hash_depends_on_tuning():
    b = _bench()
    h1 = b.kernel_sources_hash((1, 0, 2048, 1024, 8))
    assert h1 == b.kernel_sources_hash([1, 0, 2048, 1024, 8])
    assert h1 != b.kernel_sources_hash((1, 0, 1024, 1024, 8))
    assert len(h1) == 64


def test_measured_traffic_entries_are_well_formed():
    b = _bench()
    for (wl, tuning), v in b.MEASURED_TRAFFIC.items():
        assert wl == "rmat20" and len(tuning) == 5
        assert v["bytes"] > 0 and len(v["sources_sha256"]) == 64


def test_global_bin_bytes_hand_worked():
    """A 3 x 3 FP32 A with rows of 2, 0 and 1 entries and output rows of 5,
    0 and 1 entries, threshold 1: only row 0 is a global-bin row.  Its A row
    (16 B of row pointers, 2 entries of 8 B), its C row (5 entries of 8 B),
    and B = A once (4 row pointers of 8 B, 3 entries of 8 B)."""
    b = _bench()
    dense = np.array([[1.0, 0.0, 1.0], [0.0, 0.0, 0.0], [0.0, 1.0, 0.0]], dtype=np.float32)
    A = gen.from_dense(dense)
    assert A.val.dtype == np.float32
    row_nnz = np.array([5, 0, 1])
    byts, rows = b.global_bin_bytes(A, row_nnz, 1)
    assert rows == 1
    assert byts == 16 + 2 * 8 + 5 * 8 + (4 * 8 + 3 * 8)


def test_algorithmic_bytes_hand_worked():
    """FP64 A of 4 rows and 6 entries, nnz(C) = 9: A and B = A each
    5 * 8 + 6 * 12 bytes, C 5 * 8 + 9 * 12 bytes."""
    b = _bench()
    A = gen.erdos_renyi(4, 5, np.array([2, 1, 0, 3]), seed=1)
    assert A.nnz == 6 and A.val.dtype == np.float64
    assert b.algorithmic_bytes(A, 9) == 2 * (5 * 8 + 6 * 12) + (5 * 8 + 9 * 12)


def test_row_products_brute_force():
    b = _bench()
    rng = np.random.default_rng(3)
    A = gen.erdos_renyi(30, 20, rng.integers(0, 6, 30), seed=4)
    B = gen.erdos_renyi(20, 25, rng.integers(0, 7, 20), seed=5)
    blen = np.diff(B.row_ptr)
    expect = [int(sum(blen[A.col[A.row_ptr[i]:A.row_ptr[i + 1]]])) for i in range(A.nrows)]
    assert np.array_equal(b.row_products(A, B), expect)
