"""Pins of the oracle's B-row read count of Eq. (1) (``oracle.omar_distinct``)
against a hand-worked fixture, closed forms and a brute force over Python
sets; none of them calls the function under test to make its expectation."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2112_10037_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_omar.json")


def _fixture():
    d = json.load(open(GOLDEN))
    m = d["A"]
    A = gen.CSR(m["nrows"], m["ncols"], np.asarray(m["row_ptr"], np.int64), np.asarray(m["col"], np.int32),
                np.ones(len(m["col"]), np.float64))
    return d, A


@pytest.mark.parametrize("group", [1, 2, 3, 4, 5])
def test_hand_worked(group):
    d, A = _fixture()
    assert oracle.omar_distinct(A, group) == d["distinct"][str(group)]


def test_hand_worked_percent():
    d, A = _fixture()
    assert oracle.omar(A, 2) == pytest.approx(100.0 * 2 / 9, rel=1e-15)
    assert oracle.omar(A, 4) == pytest.approx(100.0 * 3 / 9, rel=1e-15)
    assert oracle.omar(A, 1) == 0.0


def _tridiagonal(n):
    rows, cols = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
    d = np.zeros((n, n))
    d[rows, cols] = 1.0
    return gen.from_dense(d)


@pytest.mark.parametrize("n,group", [(64, 1), (64, 4), (64, 8), (70, 8), (1000, 32), (33, 64)])
def test_tridiagonal_closed_form(n, group):
    # a group [g0, g1) of a tridiagonal matrix holds the columns
    # max(0, g0 - 1) .. min(n - 1, g1), all of them
    A = _tridiagonal(n)
    expect = 0
    for g0 in range(0, n, group):
        g1 = min(n, g0 + group)
        expect += min(n - 1, g1) - max(0, g0 - 1) + 1
    assert A.nnz == 3 * n - 2
    assert oracle.omar_distinct(A, group) == expect


def test_identity_and_dense():
    n = 50
    I = gen.from_dense(np.eye(n))
    for g in (1, 7, 50, 64):
        assert oracle.omar_distinct(I, g) == n          # no column repeats
    m, k = 9, 13
    D = gen.from_dense(np.ones((m, k)))
    assert oracle.omar_distinct(D, m) == k              # one group reads every column once
    assert oracle.omar_distinct(D, 1) == m * k
    assert oracle.omar(D, m) == pytest.approx(100.0 * (1 - 1 / m), rel=1e-14)


def test_empty_matrix():
    A = gen.empty(5, 7)
    assert oracle.omar_distinct(A, 3) == 0
    assert oracle.omar(A, 3) == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_brute_force(seed):
    rng = np.random.default_rng(seed)
    m, n = int(rng.integers(1, 40)), int(rng.integers(1, 30))
    pat = rng.random((m, n)) < rng.uniform(0.0, 0.5)
    pat[rng.integers(0, m)] = False                    # an empty row
    A = gen.from_dense(np.where(pat, 1.0, 0.0), pat)
    for g in (1, 2, 3, 5, 16, 100):
        sets = {}
        for i in range(m):
            s = sets.setdefault(i // g, set())
            s.update(np.nonzero(pat[i])[0].tolist())
        assert oracle.omar_distinct(A, g) == sum(len(s) for s in sets.values())
