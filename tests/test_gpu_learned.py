"""The learned output-size predictor on the GPU: network forward, gradients
and Adam against the FP64 oracle; training; and the one-pass product, whose
structure must equal the oracle's for any predictor."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2112_10037_amd import binding, gen, learned

from gpu_util import TOL, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hh = binding.Handle(0)
    yield hh
    hh.close()


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda:0") if dtype is None else t.to("cuda:0", dtype)


def _rows(seed, n=3000):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.5, (n, 8)).astype(np.float32)
    t = rng.uniform(0.0, 1.2, n).astype(np.float32)
    return x, t


def test_forward_matches_oracle(h):
    x, _ = _rows(1)
    theta = gen.mlp_init(5)
    theta[512:576] = np.random.default_rng(2).normal(0, 0.1, 64)      # nonzero biases
    p = binding.Predictor(h, theta.astype(np.float32))
    y = p.infer(_dev(x)).cpu().numpy().astype(np.float64)
    ref, _ = mlp.forward(theta.astype(np.float32).astype(np.float64), x.astype(np.float64))
    assert np.max(np.abs(y - ref) / (1 + np.abs(ref))) < 1e-5


def test_gradient_matches_oracle(h):
    """GPU FP32 gradients vs the FP64 oracle on the same weights and batch:
    relative L2 error per parameter tensor <= 1e-4."""
    x, t = _rows(3, n=5000)
    theta = gen.mlp_init(7).astype(np.float32)
    p = binding.Predictor(h, theta)
    idx = np.random.default_rng(4).integers(0, x.shape[0], 4096).astype(np.int32)
    loss, g = p.grad(_dev(x), _dev(t), _dev(idx))
    l_ref, g_ref = mlp.grad(theta.astype(np.float64), x[idx].astype(np.float64), t[idx].astype(np.float64))
    assert abs(loss - l_ref) <= 1e-5 * max(1.0, l_ref)
    o = 0
    for name, shape in mlp.SIZES:
        n = int(np.prod(shape))
        a, b = g[o:o + n].astype(np.float64), g_ref[o:o + n]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert rel <= 1e-4, (name, rel)
        o += n


def test_adam_step_matches_oracle(h):
    x, t = _rows(5)
    theta = gen.mlp_init(9).astype(np.float32)
    p = binding.Predictor(h, theta)
    idx = np.random.default_rng(6).integers(0, x.shape[0], (1, 2048)).astype(np.int32)
    p.train(_dev(x), _dev(t), _dev(idx), lr=1e-3)
    got, _ = p.get()
    _, g = mlp.grad(theta.astype(np.float64), x[idx[0]].astype(np.float64), t[idx[0]].astype(np.float64))
    ref, _, _ = mlp.adam_step(theta.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-3)
    big = np.abs(g) > 1e-6          # where the gradient's sign is not a rounding question
    assert np.max(np.abs(got[big] - ref[big])) < 2e-6


def test_training_lowers_loss_on_real_rows(h):
    import torch
    mats = [gen.erdos_renyi(3000, 3000, np.random.default_rng(1).integers(4, 33, 3000), seed=11),
            gen.rmat(12, 16 << 12, seed=12, dtype=np.float64), gen.stencil_27(14, seed=13)]
    prods = [(to_dev(M), to_dev(M)) for M in mats]
    feats, targets = learned.training_set(h, prods)
    # the GPU features and targets are the oracle's (targets from exact nnz)
    o = 0
    for M in mats:
        f_ref = oracle.features(M, M)
        t_ref = np.log2(1 + oracle.row_nnz(M, M)) / 16
        assert np.allclose(feats[o:o + M.nrows].cpu().numpy(), f_ref, rtol=2e-6, atol=2e-6)
        assert np.allclose(targets[o:o + M.nrows].cpu().numpy(), t_ref, rtol=2e-6, atol=2e-6)
        o += M.nrows
    pred, losses, delta = learned.train(h, feats, targets, steps=400, batch=2048, seed=3)
    assert losses[-20:].mean() < 0.1 * losses[:5].mean()
    assert np.isfinite(delta)
    pred.close()


@pytest.mark.parametrize("mode", ["upper", "lower", "random"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_learned_structure_exact_any_predictor(h, mode, dtype):
    """Stub predictors: 'upper' (every capacity = min(prod, n), no overflow),
    'lower' (capacity = largest B row: most rows overflow and take the exact
    fallback), 'random' weights.  The result must equal the oracle's."""
    # (matrix, whether the 'lower' stub must overflow somewhere): the 5-point
    # Laplacian has at most 25 products per row, so no row reaches the network
    mats = [(gen.rmat(11, 16 << 11, seed=21, dtype=dtype), True),
            (gen.erdos_renyi(2000, 2000, np.random.default_rng(2).integers(4, 33, 2000), seed=22,
                             dtype=dtype), True),
            (gen.stencil_27(10, seed=23, dtype=dtype), True), (gen.laplacian_2d(40, dtype=dtype), False)]
    if mode == "upper":
        params, delta = learned.fixed_capacity_params(8.0), 0.0
    elif mode == "lower":
        params, delta = learned.fixed_capacity_params(-8.0), 0.0
    else:
        params, delta = gen.mlp_init(31).astype(np.float32), 0.5
    pred = binding.Predictor(h, params)
    pred.set(None, delta)
    for M, overflows in mats:
        dM = to_dev(M)
        C, st = h.spgemm_learned(pred, dM, dM)
        got = C.to_host()
        ref = oracle.spgemm(M, M)
        oracle.compare(got.row_ptr, got.col, got.val, ref, TOL[np.dtype(dtype)])
        if mode == "upper":
            assert st["overflow_rows"] == 0
        if mode == "lower":
            assert (st["overflow_rows"] > 0) == overflows
        assert st["nnz"] == got.nnz
    pred.close()


def test_learned_matches_plain_bit_for_bit_structure(h):
    A = gen.rmat(13, 16 << 13, seed=41, dtype=np.float64)
    dA = to_dev(A)
    pred = binding.Predictor(h, learned.fixed_capacity_params(8.0))
    C1 = h.spgemm(dA, dA)
    C2, st = h.spgemm_learned(pred, dA, dA)
    import torch
    assert torch.equal(C1.row_ptr, C2.row_ptr) and torch.equal(C1.col, C2.col)
    assert st["nnz"] == C1.nnz
    pred.close()


def test_trained_network_gains_over_no_network(h):
    """Train on small members of the mixed suite and evaluate on held-out
    members: the trained capacities need less padding than the network-free
    upper bound, at a small overflow rate, with the same result."""
    import torch
    suite = gen.learned_suite()
    train_m = [m for m in suite if not m.held_out][:9]
    test_m = [m for m in suite if m.held_out][:4]
    tr = [M.build(scale_down=6) for M in train_m]
    prods = [(to_dev(M), to_dev(M)) for M in tr]
    feats, targets = learned.training_set(h, prods)
    pred, losses, delta = learned.train(h, feats, targets, steps=600, batch=4096, seed=5)
    upper = binding.Predictor(h, learned.fixed_capacity_params(8.0))
    cap_tr = cap_up = nnz = ovf = rows = 0
    for M in test_m:
        Mh = M.build(scale_down=6)
        dM = to_dev(Mh)
        C, st = h.spgemm_learned(pred, dM, dM)
        C0, st0 = h.spgemm_learned(upper, dM, dM)
        assert torch.equal(C.row_ptr, C0.row_ptr) and torch.equal(C.col, C0.col)
        cap_tr += st["sum_cap"]
        cap_up += st0["sum_cap"]
        nnz += st["nnz"]
        ovf += st["overflow_rows"]
        rows += Mh.nrows
    print(f"padding: trained {cap_tr / nnz:.3f} x nnz, upper bound {cap_up / nnz:.3f} x nnz; "
          f"overflow {ovf / rows:.4f} of rows")
    assert cap_tr < cap_up
    assert ovf <= 0.05 * rows
    # timed, at full size, on a held-out 27-point member (side 80, 512,000
    # rows), with a network trained on full-size 27-point training members
    # (the features of scaled-down members differ in their column-count
    # terms): the trained capacities keep its rows in their accumulator bins
    # where the network-free bound moves them to far larger tables
    import time
    fam = [m for m in suite if not m.held_out and m.family == "stencil27"][:3]
    fprods = []
    for Mf in fam:
        dF = to_dev(Mf.build())
        fprods.append((dF, dF))
    ffeats, ftargets = learned.training_set(h, fprods)
    del fprods
    pred.close()
    pred, _, _ = learned.train(h, ffeats, ftargets, steps=600, batch=4096, seed=5)
    M = next(m for m in suite if m.index == 59).build()
    dM = to_dev(M)

    def median_ms(fn, reps=7):
        fn()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)) * 1e3

    t_tr = median_ms(lambda: h.spgemm_learned(pred, dM, dM))
    t_up = median_ms(lambda: h.spgemm_learned(upper, dM, dM))
    t_pl = median_ms(lambda: h.spgemm(dM, dM))
    print(f"27-point side 80: trained {t_tr:.3f} ms, network-free {t_up:.3f} ms, plain {t_pl:.3f} ms")
    assert t_tr * 1.5 < t_up
    pred.close()
    upper.close()


def test_bad_batch_index_is_an_error(h):
    x, t = _rows(8, n=500)
    p = binding.Predictor(h, gen.mlp_init(3).astype(np.float32))
    idx = np.arange(256, dtype=np.int32)
    idx[17] = x.shape[0]                      # one past the end
    with pytest.raises(binding.MspError):
        p.grad(_dev(x), _dev(t), _dev(idx))
    idx[17] = 3                               # the flag was cleared
    loss, _ = p.grad(_dev(x), _dev(t), _dev(idx))
    assert np.isfinite(loss)
    p.close()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_learned_forced_spill_uses_global_bin(h, dtype):
    """Every row in the global bin (force_spill): the capacity-mode numeric
    pass runs in the sliced global kernel; with the same-bin rule each
    capacity is the row's bound, so no row overflows, and the result equals
    the oracle's."""
    params = gen.mlp_init(37).astype(np.float32)
    pred = binding.Predictor(h, params)
    pred.set(None, 0.25)
    for M in (gen.rmat(11, 16 << 11, seed=51, dtype=dtype),
              gen.erdos_renyi(1500, 1700, np.random.default_rng(4).integers(1, 20, 1500), seed=52, dtype=dtype)):
        dM = to_dev(M)
        B = M if M.nrows == M.ncols else gen.erdos_renyi(M.ncols, 900, 5, seed=53, dtype=dtype)
        dB = dM if B is M else to_dev(B)
        C, st = h.spgemm_learned(pred, dM, dB, force_spill=True)
        got = C.to_host()
        ref = oracle.spgemm(M, B)
        oracle.compare(got.row_ptr, got.col, got.val, ref, TOL[np.dtype(dtype)])
        assert st["overflow_rows"] == 0 and st["nnz"] == got.nnz
    pred.close()


@pytest.mark.slow
@pytest.mark.parametrize("index", [47, 51, 7])
def test_full_size_held_out_member_plain_and_learned(h, index):
    """A held-out member of the mixed suite at full size (index 47: 27-point
    stencil, side 49; 51: Erdos-Renyi, 2^16 rows with 4..32 per row; 7:
    R-MAT 2^16, degree 9; FP64), C = A*A through the plain path and through
    the learned one-pass path with a network trained on the GPU on small
    training members, both compared in full with the oracle."""
    suite = gen.learned_suite()
    member = next(m for m in suite if m.index == index)
    assert member.held_out
    train_m = [m for m in suite if not m.held_out][:9]
    prods = [(to_dev(M), to_dev(M)) for M in (m.build(scale_down=6) for m in train_m)]
    feats, targets = learned.training_set(h, prods)
    pred, _, _ = learned.train(h, feats, targets, steps=400, batch=4096, seed=5)
    M = member.build()
    dM = to_dev(M)
    ref = oracle.spgemm(M, M)
    plain = h.spgemm(dM, dM).to_host()
    oracle.compare(plain.row_ptr, plain.col, plain.val, ref, TOL[np.dtype(np.float64)])
    C, st = h.spgemm_learned(pred, dM, dM)
    got = C.to_host()
    oracle.compare(got.row_ptr, got.col, got.val, ref, TOL[np.dtype(np.float64)])
    assert st["nnz"] == got.nnz == plain.nnz
    print(f"member {index} ({member.family}, {M.nrows} rows): nnz(C) = {got.nnz}, "
          f"overflow rows {st['overflow_rows']}, sum cap / nnz = {st['sum_cap'] / got.nnz:.3f}")
    pred.close()


def _blocks(m, k, l, dtype=np.float64):
    """m identical rows of k entries whose B rows (l entries each) hold
    disjoint columns: prod = row nnz = k l = ncols(B), so the upper bound is
    k l and the lower bound (largest B row) l."""
    A = gen.CSR(m, k, np.arange(0, m * k + 1, k, dtype=np.int64), np.tile(np.arange(k, dtype=np.int32), m),
                np.ones(m * k, dtype))
    B = gen.CSR(k, k * l, np.arange(0, k * l + 1, l, dtype=np.int64), np.arange(k * l, dtype=np.int32),
                np.ones(k * l, dtype))
    return A, B


# (k, l, point prediction, margin delta, expected capacity).  Numeric bins of
# the tuning below: (32, 64], (64, 128], (128, 256], (256, 512], (512, 2048],
# (2048, 4096], then the global bin.  Point predictions sit half-way between
# integers, so the ceiling is the same however the FP32 network rounds.
CAPACITY_CASES = [
    (15, 100, 99.5, 0.5, 128),     # 100 * 2^0.5 = 141 is past (64, 128]: held at the bin's bound
    (15, 100, 299.5, 0.0, 300),    # bound 1500: neither twice 300 nor in its bin
    (15, 100, 599.5, 0.0, 1500),   # 600 and the bound 1500 share (512, 2048]: the bound
    (11, 50, 299.5, 0.0, 550),     # bound 550 <= 2 * 300 (bins differ): the bound
    (14, 50, 299.5, 0.0, 300),     # bound 700 > 2 * 300, bins differ: 300
    (16, 500, 5999.5, 0.0, 0),     # 8000 (the bound, within 2x) is in the global bin: exact path
]


@pytest.mark.parametrize("k,l,pt,delta,expect", CAPACITY_CASES)
def test_capacity_rule(h, k, l, pt, delta, expect):
    """The capacity rule on rows with identical bounds, one case per clause."""
    m = 300
    A, B = _blocks(m, k, l)
    pred = binding.Predictor(h, learned.fixed_capacity_params(np.log2(pt) / 16.0))
    pred.set(None, delta)
    C, st = h.spgemm_learned(pred, to_dev(A), to_dev(B), tuning=(1, 0, 4096, 1024, 8))
    assert st["sum_cap"] == m * expect
    assert st["exact_rows"] == (m if expect == 0 else 0)
    assert st["overflow_rows"] == (m if 0 < expect < k * l else 0)
    got = C.to_host()
    oracle.compare(got.row_ptr, got.col, got.val, oracle.spgemm(A, B), TOL[np.dtype(np.float64)])
    pred.close()
