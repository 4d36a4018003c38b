"""B-row sharing across the rows of a merge batch (Sec. IV-A, Fig. 3) and the
B-row read count behind OMAR (Eq. (1)): the HIP path through the C ABI
against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2112_10037_amd import binding, gen

from gpu_util import TOL, check_full, run, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hh = binding.Handle(0)
    yield hh
    hh.close()


def shared(g, k=8):
    return (1, 0, 4096, 1024, k, g)


def _csr(ref, nrows, ncols):
    rp, col, val, _ = ref
    return gen.CSR(nrows, ncols, rp, col, val)


@pytest.mark.parametrize("g", [8, 16, 32, 64])
def test_laplacian_shared_exact(h, g):
    """Integer-valued FP64 products: the merges from the LDS stage must give
    the oracle's values bit for bit.  With at most 32 rows a batch, every
    batch fits the stage and reads each distinct B row once."""
    A = gen.laplacian_2d(256)
    C = run(h, A, A, tuning=shared(g)).to_host()
    st = h.share_stats()
    rp, col, val, _ = oracle.spgemm(A, A)
    assert np.array_equal(C.row_ptr, rp) and np.array_equal(C.col, col) and np.array_equal(C.val, val)
    if g <= 32:
        assert st["a_entries"] == A.nnz                 # every row merged from the stage
        # each batch of g rows reads rows i - n, i - 1 .. i + g, i + n: about 3g + 2 of 5g
        assert st["b_rows"] < 0.7 * st["a_entries"]
        assert st["batches"] >= A.nrows // g
    else:
        assert st["b_rows"] <= st["a_entries"]


def test_laplacian_1024_shared_exact(h):
    A = gen.laplacian_2d(1024)
    C = run(h, A, A, tuning=shared(32)).to_host()
    rp, col, val, _ = oracle.spgemm(A, A)
    assert np.array_equal(C.row_ptr, rp) and np.array_equal(C.col, col) and np.array_equal(C.val, val)
    assert C.nnz == 13_611_012


def test_sharing_off_reports_nothing(h):
    A = gen.laplacian_2d(64)
    run(h, A, A)
    assert h.share_stats() == {"batches": 0, "a_entries": 0, "b_rows": 0}


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("k", [4, 8])
@pytest.mark.parametrize("g", [8, 64])
def test_er_mixed_rows(h, dtype, k, g):
    """Rows with 1..11 A entries: merge rows (at most k entries) and rows
    the merge leaves to the fallback share one batch; wide batches exceed
    the distinct-row limit and read B from global memory."""
    rng = np.random.default_rng(7)
    A = gen.erdos_renyi(3000, 512, rng.integers(0, 12, 3000), seed=8, dtype=dtype)
    B = gen.erdos_renyi(512, 700, rng.integers(0, 4, 512), seed=9, dtype=dtype)
    check_full(h, A, B, tuning=shared(g, k))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_banded_and_stencil(h, dtype):
    A = gen.banded_random(5000, 4, 40, seed=3, dtype=dtype)
    check_full(h, A, A, tuning=shared(16))
    S = gen.stencil_27(14, seed=4, dtype=dtype)
    check_full(h, S, S, tuning=shared(32))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_rmat_with_empty_rows(h, dtype):
    """Skewed rows: spans beyond the bitmap and stages that overflow fall
    back to global reads inside the same kernel."""
    A = gen.rmat(12, 8 << 12, seed=11, dtype=dtype)
    check_full(h, A, A, tuning=shared(32))


@pytest.mark.parametrize("n", [9, 16])
def test_galerkin_plain_shared(h, n):
    A, P, R = gen.galerkin_problem(n)
    check_full(h, A, P, tuning=shared(32, 4))          # 7-entry rows: the merge's fallback
    check_full(h, A, P, tuning=shared(32, 8))          # merged from the stage
    assert h.share_stats()["batches"] > 0
    AP = oracle.spgemm(A, P)
    check_full(h, R, _csr(AP, A.nrows, P.ncols), tuning=shared(32, 8))


def test_galerkin_batched_shared(h):
    sides = [int(x) for x in gen.galerkin_sizes(12, 8, 24, seed=6)]
    probs = [gen.galerkin_problem(n) for n in sides]
    pA, pP, pR = (binding.PackedBatch.from_host([x[k] for x in probs]) for k in range(3))
    plan = binding.Batch(h, pA, pP, pR, tuning=shared(32))
    plan.execute()
    for i in (0, 5, len(probs) - 1):
        A, P, R = probs[i]
        AP = oracle.spgemm(A, P)
        ref = oracle.spgemm(R, _csr(AP, A.nrows, P.ncols))
        got = plan.result(i).to_host()
        oracle.compare(got.row_ptr, got.col, got.val, ref, TOL[np.dtype(np.float64)])
    plan.close()


def test_shared_tuning_validation(h):
    A = gen.laplacian_2d(16)
    with pytest.raises(binding.MspError):
        h.set_tuning((1, 0, 4096, 1024, 8, 4))          # below 8 rows
    with pytest.raises(binding.MspError):
        h.set_tuning((1, 0, 4096, 1024, 8, 65))
    js = binding.tuning_to_json(shared(24))
    assert binding.tuning_from_json(js) == shared(24)
    check_full(h, A, A, tuning=shared(24))


# ---- the B-row read count of Eq. (1) ---------------------------------------

def _omar_cases():
    rng = np.random.default_rng(5)
    pat = rng.random((37, 29)) < 0.3
    pat[[3, 17]] = False                                 # empty rows
    return [
        ("laplacian", gen.laplacian_2d(40)),
        ("stencil27", gen.stencil_27(12, seed=2)),
        ("er", gen.erdos_renyi(4096, 4096, 8, seed=0)),
        ("rmat", gen.rmat(12, 16 << 12, seed=3, dtype=np.float32)),
        ("random", gen.from_dense(np.where(pat, 1.0, 0.0), pat)),
    ]


@pytest.mark.parametrize("group", [1, 2, 3, 8, 32, 64, 4096])
def test_omar_matches_oracle(h, group):
    for name, A in _omar_cases():
        dA = to_dev(A)
        assert h.omar_distinct(dA, group) == oracle.omar_distinct(A, group), (name, group)


def test_omar_edges(h):
    E = gen.empty(6, 9)
    assert h.omar_distinct(to_dev(E), 4) == 0
    A = gen.laplacian_2d(8)
    dA = to_dev(A)
    with pytest.raises(binding.MspError):
        h.omar_distinct(dA, 0)
    with pytest.raises(binding.MspError):
        h.omar_distinct(dA, 4097)
    assert h.omar(dA, 1) == 0.0
    assert h.omar(dA, 64) == pytest.approx(oracle.omar(A, 64), rel=1e-12)
