"""The rest of the C-ABI boundary on the GPU: predictor checkpoints, the
single-product autotuner, and the failing-allocator path."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2112_10037_amd import binding, gen, learned

from gpu_util import TOL, check_full, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hh = binding.Handle(0)
    yield hh
    hh.close()


def test_predictor_save_load_resumes_training(h):
    """Save after some Adam steps, train on, reload the checkpoint into a
    fresh predictor and train the same steps again: both runs end with the
    same parameters bit for bit (the blob carries the moments and step)."""
    import torch
    A = gen.rmat(11, 12 << 11, seed=41, dtype=np.float64)
    dA = to_dev(A)
    feats, targets = h.training_rows(dA, dA)
    rng = np.random.default_rng(0)
    idx = torch.from_numpy(rng.integers(0, feats.shape[0], (20, 256)).astype(np.int32)).cuda()
    p0 = gen.mlp_init(1).astype(np.float32)
    P = binding.Predictor(h, p0)
    try:
        P.train(feats, targets, idx[:10])
        P.set(P.get()[0], 1.5)
        blob = P.save()
        assert len(blob) == binding.BLOB_BYTES
        params, delta, m, v, step = binding.blob_unpack(blob)
        assert delta == 1.5 and step == 10 and np.any(m != 0) and np.all(v >= 0)
        assert np.array_equal(params, P.get()[0])
        P.train(feats, targets, idx[10:])
        end_a = P.get()[0]
    finally:
        P.close()
    Q = binding.Predictor(h, p0)
    try:
        Q.load(blob)
        assert Q.get()[1] == 1.5 and np.array_equal(Q.get()[0], params)
        Q.train(feats, targets, idx[10:])
        assert np.array_equal(Q.get()[0], end_a)
        with pytest.raises(binding.MspError) as e:
            Q.load(blob[:-8] + bytes(8))
        assert e.value.name == "MSP_ERR_INVALID_ARG"
        assert np.array_equal(Q.get()[0], end_a)          # unchanged by the refused blob
    finally:
        Q.close()


def test_autotune_single_product(h):
    A = gen.rmat(12, 12 << 12, seed=15, dtype=np.float64)
    dA = to_dev(A)
    cand = [(1, 0, 4096, 1024, 8), (2, 0, 4096, 128, 4), (1, 1, 1024, 64, -1)]
    before = h.get_tuning()
    best, times = h.autotune(dA, dA, cand, reps=3)
    assert best in cand and len(times) == 3 and all(np.isfinite(t) and t > 0 for t in times)
    assert best == cand[int(np.argmin(times))]
    assert h.get_tuning() == before
    assert not h._live                         # every C of the timed calls released
    check_full(h, A, A, tuning=best)


class _CountingHandle(binding.Handle):
    """Allocator callbacks that record every block and fail the requests
    whose size the test names."""

    def __init__(self, fail_above):
        self.fail_above = fail_above
        self.allocs, self.frees = [], []
        super().__init__(0)

    def _alloc(self, ctx, nbytes, stream):
        if nbytes > self.fail_above:
            return None
        p = super()._alloc(ctx, nbytes, stream)
        if p:
            self.allocs.append(p)
        return p

    def _free(self, ctx, ptr, stream):
        self.frees.append(ptr)
        super()._free(ctx, ptr, stream)


@pytest.mark.parametrize("own_row_ptr", [False, True])
def test_failing_allocator_gives_oom_and_leaks_nothing(own_row_ptr):
    """The allocation of C's columns and values fails: MSP_ERR_OOM, C's
    pointers null, every block the library obtained released; the handle
    then computes the next product normally."""
    A = gen.erdos_renyi(3000, 3000, 7, seed=2)
    m = A.nrows
    hh = _CountingHandle(fail_above=(m + 1) * 8)      # row_ptr fits, C does not
    try:
        dA = to_dev(A)
        a = dA.c()
        out = binding.c_csr_out()
        keep = None
        if own_row_ptr:
            import torch
            keep = torch.empty(m + 1, dtype=torch.int64, device="cuda")
            out.row_ptr = keep.data_ptr()
        st = hh._lib.msp_spgemm(hh._h, ctypes.byref(a), ctypes.byref(a), ctypes.byref(out), None)
        assert binding.STATUS[st] == "MSP_ERR_OOM", hh._lib.msp_last_error()
        assert b"allocation of C" in hh._lib.msp_last_error()
        assert not out.col and not out.val
        if own_row_ptr:
            assert out.row_ptr == keep.data_ptr()        # the caller's buffer is left alone
        else:
            assert not out.row_ptr
        assert sorted(hh.allocs) == sorted(hh.frees)     # nothing leaked
        assert not hh._live
        hh.sync()
        hh.fail_above = 1 << 62
        C = hh.spgemm(dA, dA)
        host = C.to_host()
        oracle.compare(host.row_ptr, host.col, host.val, oracle.spgemm(A, A), TOL[np.dtype(np.float64)])
    finally:
        hh.close()
