"""Batched products in one graph launch, against the oracle problem by
problem: single-stage batches of mixed shapes (every bin kind), Galerkin
triple products R (A P), replays with new values, detection of structure
changes, and the autotuner."""
import numpy as np
import pytest

import oracle
from paper_2112_10037_amd import binding, gen

from gpu_util import TOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hh = binding.Handle(0)
    yield hh
    hh.close()


def _csr(ref, nrows, ncols):
    rp, col, val, _ = ref
    return gen.CSR(nrows, ncols, rp, col, val)


def _check(Cd, ref, dtype):
    got = Cd.to_host()
    return oracle.compare(got.row_ptr, got.col, got.val, ref, TOL[np.dtype(dtype)])


def _hub(n, seed, dtype):
    """n x n with a few dense rows (long B rows and long A rows)."""
    rng = np.random.default_rng(seed)
    d = np.zeros((n, n), dtype=bool)
    for i in range(n):
        d[i, rng.choice(n, size=int(rng.integers(1, 6)), replace=False)] = True
    d[rng.choice(n, 3, replace=False)] = rng.random((3, n)) < 0.7
    d[:, rng.choice(n, 2, replace=False)] = True
    return gen.from_dense(np.where(d, rng.uniform(-1, 1, (n, n)), 0.0).astype(dtype), d)


def _mixed(dtype, seed=3):
    """Problems of every bin kind: short rows, hash rows, hub rows, wide
    spill rows, an empty problem and a 1 x 1 problem."""
    A, B = [], []
    rng = np.random.default_rng(seed)
    A.append(gen.erdos_renyi(700, 500, rng.integers(1, 9, 700), seed=1, dtype=dtype))
    B.append(gen.erdos_renyi(500, 900, rng.integers(1, 9, 500), seed=2, dtype=dtype))
    L = gen.laplacian_2d(30, dtype=dtype)
    A.append(L), B.append(L)
    R = gen.rmat(11, 16 << 11, seed=4, dtype=dtype)
    A.append(R), B.append(R)
    A.append(gen.empty(0, 40, dtype)), B.append(gen.erdos_renyi(40, 40, 3, seed=5, dtype=dtype))
    H = _hub(600, 6, dtype)
    A.append(H), B.append(H)
    S = gen.stencil_27(9, seed=7, dtype=dtype)
    A.append(S), B.append(S)
    A.append(gen.from_dense(np.array([[2.0]], dtype=dtype))), B.append(gen.from_dense(np.array([[3.0]], dtype=dtype)))
    W = gen.erdos_renyi(64, 1 << 15, 6000, seed=8, dtype=dtype)        # long rows over wide B: global path
    Wb = gen.erdos_renyi(1 << 15, 1 << 15, 4, seed=9, dtype=dtype)
    A.append(W), B.append(Wb)
    return A, B


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batch_single_stage_matches_oracle(h, dtype):
    A, B = _mixed(dtype)
    pa, pb = binding.PackedBatch.from_host(A), binding.PackedBatch.from_host(B)
    plan = binding.Batch(h, pa, pb)
    info = plan.info()
    assert info["nstage"] == 1
    assert info["num_bins"][0] >= 3 and info["sym_bins"][0] >= 3
    plan.execute()
    plan.sync()
    worst = 0.0
    for p in range(len(A)):
        worst = max(worst, _check(plan.result(p), oracle.spgemm(A[p], B[p]), dtype))
    print(f"max |c-o|/bound = {worst:.3e}")
    plan.close()


def test_batch_agrees_with_single_products_on_views(h):
    """The plain call on a problem's view of the packed batch gives the same
    structure (and values within the bound) as the batch."""
    import torch
    A, B = _mixed(np.float64, seed=11)
    pa, pb = binding.PackedBatch.from_host(A), binding.PackedBatch.from_host(B)
    plan = binding.Batch(h, pa, pb)
    plan.execute()
    for p in range(len(A)):
        Cb = plan.result(p)
        Cs = h.spgemm(pa.view(p), pb.view(p))
        assert torch.equal(Cb.row_ptr, Cs.row_ptr) and torch.equal(Cb.col, Cs.col), p
        ref = oracle.spgemm(A[p], B[p])
        _check(Cs, ref, np.float64)
    plan.close()


def test_galerkin_batch_exact(h):
    """R (A P) for 7-point Laplacians and aggregation prolongators: integer
    values, so structure and values are exact; even sides give 4 L_{n/2}."""
    sides = [3, 4, 5, 8, 9, 12, 16, 7, 6, 10, 13, 2]
    probs = [gen.galerkin_problem(n) for n in sides]
    A = [a for a, _, _ in probs]
    P = [p for _, p, _ in probs]
    R = [r for _, _, r in probs]
    pA, pP, pR = (binding.PackedBatch.from_host(x) for x in (A, P, R))
    plan = binding.Batch(h, pA, pP, pR)
    assert plan.info()["nstage"] == 2
    plan.execute()
    for i, n in enumerate(sides):
        AP = oracle.spgemm(A[i], P[i])
        ref = oracle.spgemm(R[i], _csr(AP, A[i].nrows, P[i].ncols))
        got = plan.result(i).to_host()
        assert np.array_equal(got.row_ptr, ref[0]) and np.array_equal(got.col, ref[1])
        assert np.array_equal(got.val, ref[2]), n
        if n % 2 == 0:
            L = gen.laplacian_3d(n // 2)
            assert np.array_equal(got.col, L.col) and np.array_equal(got.val, 4 * L.val)
    plan.close()


def test_replay_reads_new_values(h):
    import torch
    sides = [4, 6, 9, 5]
    probs = [gen.galerkin_problem(n) for n in sides]
    A = [a for a, _, _ in probs]
    P = [p for _, p, _ in probs]
    R = [r for _, _, r in probs]
    pA, pP, pR = (binding.PackedBatch.from_host(x) for x in (A, P, R))
    plan = binding.Batch(h, pA, pP, pR)
    for rep, scale in enumerate([1.0, -2.5, 0.5]):
        pA.val.copy_(torch.from_numpy(np.concatenate([a.val for a in A]) * scale).to(pA.val.device))
        plan.execute()
        for i in range(len(sides)):
            As = gen.CSR(A[i].nrows, A[i].ncols, A[i].row_ptr, A[i].col, A[i].val * scale)
            AP = oracle.spgemm(As, P[i])
            ref = oracle.spgemm(R[i], _csr(AP, A[i].nrows, P[i].ncols))
            _check(plan.result(i), ref, np.float64)
    plan.close()


def test_structure_change_is_reported(h):
    """A replay whose rows would need a bin kernel the plan lacks, or whose
    output outgrows the plan's arena, raises and produces nothing; a new
    plan then works."""
    import torch
    n = 512
    rng = np.random.default_rng(5)
    # B: every row one entry in column 0; A: 2 entries per row -> 1 output per row
    Bh = gen.CSR(n, n, np.arange(n + 1, dtype=np.int64), np.zeros(n, np.int32), np.ones(n))
    Ah = gen.erdos_renyi(n, n, 2, seed=12)
    pa, pb = binding.PackedBatch.from_host([Ah]), binding.PackedBatch.from_host([Bh])
    plan = binding.Batch(h, pa, pb)
    plan.execute()
    plan.sync()
    # distinct columns in B: twice the output, same bins -> capacity error
    pb.col.copy_(torch.arange(n, dtype=torch.int32, device=pb.col.device))
    plan.execute()
    with pytest.raises(binding.MspError, match="outgrew"):
        plan.sync()
    # B row 0 made long (same nnz, so B's row 1.. lose their entries) -> bin error
    long_rp = np.zeros(n + 1, dtype=np.int64)
    long_rp[1:] = n
    pb.row_ptr.copy_(torch.from_numpy(long_rp).to(pb.row_ptr.device))
    a_col = np.zeros(2 * n, dtype=np.int32)
    a_col[1::2] = 1                                     # every A row: columns 0 and 1 (sorted, unique)
    pa.col.copy_(torch.from_numpy(a_col).to(pa.col.device))
    plan.execute()
    with pytest.raises(binding.MspError, match="structure changed"):
        plan.sync()
    plan.close()
    # a fresh plan of the new structure is right
    Bn = gen.CSR(n, n, long_rp, np.arange(n, dtype=np.int32), np.ones(n))
    An = gen.CSR(n, n, Ah.row_ptr, a_col, np.asarray(Ah.val))
    plan2 = binding.Batch(h, pa, pb)
    plan2.execute()
    _check(plan2.result(0), oracle.spgemm(An, Bn), np.float64)
    plan2.close()
    del rng


def test_autotune_picks_a_candidate(h):
    sides = [int(x) for x in gen.galerkin_sizes(16, 8, 20, seed=3)]
    probs = [gen.galerkin_problem(n) for n in sides]
    pA, pP, pR = (binding.PackedBatch.from_host([x[k] for x in probs]) for k in range(3))
    cands = [(1, 0, 4096, 128, 8), (1, 0, 4096, 128, 4), (2, 1, 1024, 64, -1)]
    best, times = binding.autotune(h, pA, pP, pR, cands, reps=3)
    assert best in cands
    assert all(np.isfinite(times)) and times[cands.index(best)] == min(times)
    js = binding.tuning_to_json(best)
    assert binding.tuning_from_json(js) == best
    plan = binding.Batch(h, pA, pP, pR, tuning=best)
    plan.execute()
    i = 1
    AP = oracle.spgemm(probs[i][0], probs[i][1])
    ref = oracle.spgemm(probs[i][2], _csr(AP, probs[i][0].nrows, probs[i][1].ncols))
    got = plan.result(i).to_host()
    assert np.array_equal(got.col, ref[1]) and np.array_equal(got.val, ref[2])
    plan.close()


def test_batch_full_merge_batches(h):
    """Four problems of 4,096 rows with at most 4 outputs per row (16,384
    rows in all): every merge batch takes all 64 of its rows."""
    rng = np.random.default_rng(31)
    A = [gen.erdos_renyi(4096, 2048, rng.integers(1, 5, 4096), seed=40 + i) for i in range(4)]
    P = [gen.aggregation_prolongator(n)[0] for n in (13, 13, 13, 13)]          # 2197 x 343
    P = [gen.CSR(2048, 343, p.row_ptr[:2049], p.col[:2048], p.val[:2048]) for p in P]
    pa, pp = binding.PackedBatch.from_host(A), binding.PackedBatch.from_host(P)
    plan = binding.Batch(h, pa, pp)
    plan.execute()
    for i in range(4):
        _check(plan.result(i), oracle.spgemm(A[i], P[i]), np.float64)
    plan.close()


@pytest.mark.slow
def test_galerkin_512_full_batch_against_oracle(h):
    """The full batched workload: 512 Galerkin products R (A P), 7-point
    Laplacians with sides n ~ U{16..64} (seed 5), 2x2x2 aggregation, FP64,
    planned and replayed as one graph; every problem's result is compared
    with the oracle (two oracle products per distinct side; problems of one
    side are the same matrices).  Values are integers: exact equality."""
    from paper_2112_10037_amd import batch
    sides = gen.galerkin_sizes(512, 16, 64, seed=5)
    pA, pP, pR = batch.galerkin_batch(sides)
    plan = binding.Batch(h, pA, pP, pR)
    plan.execute()
    plan.sync()
    refs = {}
    A, P, R = batch.galerkin_host(sides)
    for p, n in enumerate(sides):
        n = int(n)
        if n not in refs:
            AP = oracle.spgemm(A[p], P[p])
            refs[n] = oracle.spgemm(R[p], _csr(AP, A[p].nrows, P[p].ncols))
        ref = refs[n]
        got = plan.result(p).to_host()
        assert np.array_equal(got.row_ptr, ref[0]) and np.array_equal(got.col, ref[1]), (p, n)
        assert np.array_equal(got.val, ref[2]), (p, n)
    plan.close()


def test_uneven_batch_work_queue(h):
    """Problem sides 2..64 in one batch (8 to 262,144 rows each): the numeric
    merge's waves draw row blocks from the shared work queue; every problem
    is checked against the oracle, and the static split (one row range per
    wave) and a small ticket give the same results bit for bit."""
    rng = np.random.default_rng(17)
    sides = [2, 64, 3, 5, 63, 2, 17, 40] + [int(x) for x in rng.integers(2, 65, 16)]
    probs = [gen.galerkin_problem(n) for n in sides]
    pA, pP, pR = (binding.PackedBatch.from_host([x[k] for x in probs]) for k in range(3))
    plans = {q: binding.Batch(h, pA, pP, pR, queue_rows=q) for q in (0, -1, 64)}
    for plan in plans.values():
        plan.execute()
    for i, (A, P, R) in enumerate(probs):
        AP = oracle.spgemm(A, P)
        ref = oracle.spgemm(R, _csr(AP, A.nrows, P.ncols))
        got = plans[0].result(i).to_host()
        oracle.compare(got.row_ptr, got.col, got.val, ref, TOL[np.dtype(np.float64)])
        for q in (-1, 64):
            other = plans[q].result(i).to_host()
            assert np.array_equal(other.row_ptr, got.row_ptr) and np.array_equal(other.col, got.col)
            assert np.array_equal(other.val, got.val)
    for plan in plans.values():
        plan.close()


def test_work_queue_rows_validation(h):
    probs = [gen.galerkin_problem(n) for n in (4, 5)]
    pA, pP, pR = (binding.PackedBatch.from_host([x[k] for x in probs]) for k in range(3))
    for bad in (32, 100, 65600, -2):
        with pytest.raises(binding.MspError):
            binding.Batch(h, pA, pP, pR, queue_rows=bad)
    plan = binding.Batch(h, pA, pP, pR, queue_rows=65536)
    plan.execute()
    A, P, R = probs[1]
    AP = oracle.spgemm(A, P)
    ref = oracle.spgemm(R, _csr(AP, A.nrows, P.ncols))
    got = plan.result(1).to_host()
    assert np.array_equal(got.col, ref[1]) and np.array_equal(got.val, ref[2])
    plan.close()
