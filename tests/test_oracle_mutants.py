"""Plant plausible mistakes in a copy of the C oracle (on the CPU) and check
that the pins catch each one: this shows the pins constrain the oracle."""
import os

import numpy as np
import pytest

import oracle
from paper_2112_10037_amd import gen

SRC = os.path.join(os.path.dirname(oracle.__file__), "spgemm_oracle.c")

MUTANTS = {
    "sign_of_add": ("acc[j] = acc[j] + t;", "acc[j] = acc[j] - t;"),
    "dropped_first_term": ("double t = a * b;", "double t = (q == b_ptr[k]) ? 0.0 : a * b;"),
    "wrong_a_index": ("double a = load_val(a_val, is_f32, p);",
                      "double a = load_val(a_val, is_f32, a_ptr[i]);"),
    "no_sort": ("qsort(list,", "if (0) qsort(list,"),
    "stale_marker": ("if (mark[j] != i) {\n                            mark[j] = i;\n                            acc[j]",
                     "if (mark[j] < 0) {\n                            mark[j] = i;\n                            acc[j]"),
    "transposed_b": ("int32_t j = b_col[q];\n                        double b",
                     "int32_t j = (int32_t)(q - b_ptr[k]) % (int32_t)ncols_b;\n                        double b"),
}


def _pins_pass() -> bool:
    """A compact subset of the pins; True if all hold."""
    try:
        A = gen.from_dense(np.array([[1, 0, 2], [0, 3, 0], [4, 0, 5.0]]))
        rp, col, val, _ = oracle.spgemm(A, A)
        if rp.tolist() != [0, 2, 3, 5] or col.tolist() != [0, 2, 1, 0, 2] \
                or val.tolist() != [9.0, 12.0, 9.0, 24.0, 33.0]:
            return False
        rng = np.random.default_rng(1)
        for _ in range(3):
            pa = rng.random((20, 17)) < 0.3
            pb = rng.random((17, 23)) < 0.3
            Ad = np.where(pa, rng.uniform(-1, 1, pa.shape), 0.0)
            Bd = np.where(pb, rng.uniform(-1, 1, pb.shape), 0.0)
            A, B = gen.from_dense(Ad, pa), gen.from_dense(Bd, pb)
            rp, col, val, bnd = oracle.spgemm(A, B)
            pat = (pa.astype(int) @ pb.astype(int)) > 0
            r, c = np.nonzero(pat)
            if rp[-1] != pat.sum() or not np.array_equal(col, c):
                return False
            if not np.all(np.abs(val - (Ad @ Bd)[r, c]) <= 1e-13 * (np.abs(Ad) @ np.abs(Bd))[r, c]):
                return False
        return True
    except (AssertionError, RuntimeError, ValueError, IndexError):
        return False


def test_pins_pass_on_real_oracle():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = oracle.build(str(path), str(tmp_path / "libmutant.so"))
    prev = oracle.use_library(so)
    try:
        assert not _pins_pass(), f"pins did not catch mutant {name}"
    finally:
        oracle.use_library(None)
