"""Pin of the oracle's predictor inputs (``oracle.features``) against a
hand-worked fixture, and planted mistakes in a copy of that function (on the
CPU) that the fixture must reject.

The fixture (tests/golden/hand_features.json) states the per-row statistics
and the eight inputs as literal numbers worked out by hand from their
definitions; nothing in it comes from either implementation.
"""
import inspect
import json
import os
import textwrap

import numpy as np
import pytest

import oracle
from paper_2112_10037_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_features.json")


def _fixture():
    d = json.load(open(GOLDEN))
    mk = lambda m: gen.CSR(m["nrows"], m["ncols"], np.asarray(m["row_ptr"], np.int64),
                           np.asarray(m["col"], np.int32),
                           np.ones(len(m["col"]), np.float64))
    return d, mk(d["A"]), mk(d["B"])


def test_fixture_is_canonical():
    d, A, B = _fixture()
    A.check()
    B.check()


def test_row_stats_match_hand_worked():
    d, A, B = _fixture()
    s = oracle.row_stats(A, B)
    for k, v in d["stats"].items():
        assert s[k].tolist() == v, k


def _agrees(f, expect) -> bool:
    return f.shape == expect.shape and bool(np.all(np.abs(f - expect) <= 1e-15))


def test_features_match_hand_worked():
    d, A, B = _fixture()
    f = oracle.features(A, B)
    assert _agrees(f, np.asarray(d["features"], np.float64)), f - np.asarray(d["features"])


def test_features_of_empty_product():
    A = gen.empty(3, 4)
    B = gen.empty(4, 7)
    f = oracle.features(A, B)
    assert f.shape == (3, 8)
    assert np.all(f[:, [0, 1, 2, 3, 4, 6, 7]] == 0.0)
    assert np.all(f[:, 5] == 0.1875)          # log2(1 + 7) / 16


# Plausible mistakes in the feature code: a wrong mean, span or scale, or a
# swapped column.  Each is planted in a copy of the function's source.
MUTANTS = {
    "mean_over_ncols": ("mean_b = np.divide(prod, nnz_a,", "mean_b = np.divide(prod, float(B.ncols) + 0 * nnz_a,"),
    "scale_8": ("f[:, 0] = np.log2(1.0 + nnz_a) / 16.0", "f[:, 0] = np.log2(1.0 + nnz_a) / 8.0"),
    "no_plus_one": ("f[:, 1] = np.log2(1.0 + prod) / 16.0", "f[:, 1] = np.log2(np.maximum(prod, 1.0)) / 16.0"),
    "span_over_nrows": ('f[:, 7] = s["span"] / n', 'f[:, 7] = s["span"] / max(A.nrows, 1)'),
    "min_max_swapped": ('f[:, 2] = np.log2(1.0 + s["min_b"]) / 16.0',
                        'f[:, 2] = np.log2(1.0 + s["max_b"]) / 16.0'),
    "no_clamp": ("f[:, 6] = np.minimum(1.0, prod / n)", "f[:, 6] = prod / n"),
    "ncols_of_a": ("f[:, 5] = np.log2(1.0 + float(B.ncols)) / 16.0",
                   "f[:, 5] = np.log2(1.0 + float(A.ncols)) / 16.0"),
}


def _mutated(name):
    old, new = MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(oracle.features))
    assert src.count(old) == 1, name
    ns = {"np": np, "row_stats": oracle.row_stats}
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), ns)
    return ns["features"]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_fixture_catches_mutant(name):
    d, A, B = _fixture()
    f = _mutated(name)(A, B)
    assert not _agrees(f, np.asarray(d["features"], np.float64)), f"fixture did not catch {name}"
