"""Thin ctypes binding of libmsp.so (the C ABI in include/msp.h).

Argument marshalling only: every step of the product runs in the library's
HIP kernels.  PyTorch provides device memory (input copies and the output
arrays, through the allocator callback) and the stream.  If the library is
missing or cannot be loaded, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsp.so")

MSP_F32, MSP_F64 = 0, 1
STATUS = {0: "MSP_OK", 1: "MSP_ERR_INVALID_ARG", 2: "MSP_ERR_SHAPE", 3: "MSP_ERR_DTYPE",
          4: "MSP_ERR_UNSORTED_OR_DUP", 5: "MSP_ERR_OOM", 6: "MSP_ERR_HIP",
          7: "MSP_ERR_INDEX_OVERFLOW", 8: "MSP_ERR_UNSUPPORTED"}


class MspError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class c_csr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("dtype", ctypes.c_int)]


class c_csr_out(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("dtype", ctypes.c_int)]


class c_tuning(ctypes.Structure):
    _fields_ = [("hash_scale", ctypes.c_int32), ("group_scale", ctypes.c_int32),
                ("spill_nnz", ctypes.c_int32), ("block_rows", ctypes.c_int32),
                ("merge_k", ctypes.c_int32), ("share_g", ctypes.c_int32)]


def _tuple(t: "c_tuning"):
    """A tuning as a tuple: its five fields, and share_g sixth when sharing
    is on (a five-field tuple leaves it at the default, off)."""
    base = (t.hash_scale, t.group_scale, t.spill_nnz, t.block_rows, t.merge_k)
    return base + (t.share_g,) if t.share_g > 0 else base


class c_share_stats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_int64), ("a_entries", ctypes.c_int64), ("b_rows", ctypes.c_int64)]


class c_opts(ctypes.Structure):
    _fields_ = [("validate", ctypes.c_int32), ("force_spill", ctypes.c_int32),
                ("tuning", c_tuning), ("queue_rows", ctypes.c_int32)]


class c_train_opts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class c_learned_stats(ctypes.Structure):
    _fields_ = [("overflow_rows", ctypes.c_int64), ("sum_cap", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("exact_rows", ctypes.c_int64)]


class c_batch_csr(ctypes.Structure):
    _fields_ = [("nprob", ctypes.c_int32), ("row_start", ctypes.c_void_p), ("ncols", ctypes.c_void_p),
                ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("dtype", ctypes.c_int)]


class c_batch_stats(ctypes.Structure):
    _fields_ = [("nstage", ctypes.c_int32), ("rows", ctypes.c_int64 * 2), ("nnz", ctypes.c_int64 * 2),
                ("sym_bins", ctypes.c_int32 * 2), ("num_bins", ctypes.c_int32 * 2)]


NUM_PHASES = 9
PHASES = ["row_stats", "symbolic", "scan", "numeric", "predict", "fallback", "compact", "batch", "global_bin"]


class c_profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * NUM_PHASES), ("count", ctypes.c_int64 * NUM_PHASES)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

_lib = None

# (name, restype, argtypes) of every symbol include/msp.h declares
SIGNATURES = [
    ("msp_create", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p]),
    ("msp_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("msp_set_stream", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("msp_set_allocator", ctypes.c_int, [ctypes.c_void_p, ALLOC_FN, FREE_FN, ctypes.c_void_p]),
    ("msp_set_tuning", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_tuning)]),
    ("msp_get_tuning", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_tuning)]),
    ("msp_spgemm", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_csr), ctypes.POINTER(c_csr),
                                  ctypes.POINTER(c_csr_out), ctypes.POINTER(c_opts)]),
    ("msp_sync", ctypes.c_int, [ctypes.c_void_p]),
    ("msp_spgemm_noalloc", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_csr), ctypes.POINTER(c_csr),
                                          ctypes.POINTER(c_csr_out), ctypes.c_int64, ctypes.POINTER(c_opts)]),
    ("msp_spgemm_symbolic", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_csr), ctypes.POINTER(c_csr),
                                           ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(c_opts)]),
    ("msp_row_features", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_csr), ctypes.POINTER(c_csr),
                                        ctypes.c_void_p, ctypes.c_void_p]),
    ("msp_predictor_create", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    ("msp_predictor_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("msp_predictor_get", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_float)]),
    ("msp_predictor_set", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float]),
    ("msp_predictor_save", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.POINTER(ctypes.c_size_t)]),
    ("msp_predictor_load", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    ("msp_predictor_blob_pack", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float,
                                               ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t,
                                               ctypes.POINTER(ctypes.c_size_t)]),
    ("msp_predictor_blob_unpack", ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                                 ctypes.POINTER(ctypes.c_int64)]),
    ("msp_predictor_train", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(c_train_opts), ctypes.c_void_p]),
    ("msp_predictor_grad", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    ("msp_predictor_infer", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_void_p]),
    ("msp_predictor_calibrate", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_int64, ctypes.c_double]),
    ("msp_training_rows", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_csr), ctypes.POINTER(c_csr),
                                         ctypes.c_void_p, ctypes.c_void_p]),
    ("msp_spgemm_learned", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(c_csr),
                                          ctypes.POINTER(c_csr), ctypes.POINTER(c_csr_out),
                                          ctypes.POINTER(c_opts), ctypes.POINTER(c_learned_stats)]),
    ("msp_batch_create", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_batch_csr), ctypes.POINTER(c_batch_csr),
                                        ctypes.POINTER(c_batch_csr), ctypes.POINTER(c_opts),
                                        ctypes.POINTER(ctypes.c_void_p)]),
    ("msp_batch_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("msp_batch_execute", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("msp_batch_sync", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("msp_batch_result", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(c_csr)]),
    ("msp_batch_copy_result", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                             ctypes.POINTER(c_csr_out)]),
    ("msp_batch_info", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_batch_stats)]),
    ("msp_batch_autotune", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_batch_csr),
                                          ctypes.POINTER(c_batch_csr), ctypes.POINTER(c_batch_csr),
                                          ctypes.POINTER(c_tuning), ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(c_tuning), ctypes.POINTER(ctypes.c_double)]),
    ("msp_autotune", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_csr), ctypes.POINTER(c_csr),
                                    ctypes.POINTER(c_tuning), ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(c_tuning), ctypes.POINTER(ctypes.c_double)]),
    ("msp_omar", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_csr), ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_int64)]),
    ("msp_share_stats_get", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_share_stats)]),
    ("msp_tuning_to_json", ctypes.c_int, [ctypes.POINTER(c_tuning), ctypes.c_char_p, ctypes.c_size_t]),
    ("msp_tuning_from_json", ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(c_tuning)]),
    ("msp_profile_enable", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("msp_profile_get", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(c_profile)]),
    ("msp_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("msp_last_error", ctypes.c_char_p, []),
    ("msp_version", ctypes.c_int, []),
]


def load():
    """Load libmsp.so (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2112_10037_amd/build.py "
                              "(or __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != 0:
        raise MspError(rc, load().msp_last_error().decode())


# ---------------------------------------------------------------------------
# device matrices
# ---------------------------------------------------------------------------

@dataclass
class DeviceCSR:
    """CSR on the GPU: int64 row_ptr, int32 col, f32/f64 val torch tensors."""
    nrows: int
    ncols: int
    row_ptr: "object"
    col: "object"
    val: "object"

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @property
    def dtype_code(self) -> int:
        import torch
        return MSP_F64 if self.val.dtype == torch.float64 else MSP_F32

    @classmethod
    def from_host(cls, m, device="cuda") -> "DeviceCSR":
        import torch
        return cls(int(m.nrows), int(m.ncols),
                   torch.from_numpy(np.ascontiguousarray(m.row_ptr, np.int64)).to(device),
                   torch.from_numpy(np.ascontiguousarray(m.col, np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(m.val)).to(device))

    def to_host(self):
        from .gen import CSR
        return CSR(self.nrows, self.ncols, self.row_ptr.cpu().numpy(), self.col.cpu().numpy(),
                   self.val.cpu().numpy())

    def c(self) -> c_csr:
        return c_csr(self.nrows, self.ncols, self.nnz, self.row_ptr.data_ptr(),
                     self.col.data_ptr() if self.nnz else None,
                     self.val.data_ptr() if self.nnz else None, self.dtype_code)


def _opts(validate=False, force_spill=False, tuning=None, queue_rows=0) -> c_opts:
    t = c_tuning(*(tuning or (0, 0, 0, 0, 0)))
    return c_opts(int(bool(validate)), int(bool(force_spill)), t, int(queue_rows))


class Handle:
    """One library handle on one device, queueing work on torch's current
    stream (or the stream given)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._lib = load()
        self.device = device
        self._torch = torch
        self._h = ctypes.c_void_p()
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self._stream = s
        _check(self._lib.msp_create(ctypes.byref(self._h), device, ctypes.c_void_p(s.cuda_stream)))
        self._live = {}
        self._same_stream = None
        self._alloc_cb = ALLOC_FN(self._alloc)
        self._free_cb = FREE_FN(self._free)
        _check(self._lib.msp_set_allocator(self._h, self._alloc_cb, self._free_cb, None))

    # allocator callbacks: torch tensors kept alive until handed out or freed
    def _alloc(self, ctx, nbytes, stream):
        try:
            t = self._torch.empty(max(int(nbytes), 1), dtype=self._torch.uint8,
                                  device=f"cuda:{self.device}")
        except RuntimeError:
            return None
        # torch files the block under its current stream; when the library
        # queues on another one, the block is also marked in use there, so
        # that it is not handed out again before that stream's work is done
        # (the product entry points compare the streams before the call,
        # while the GPU may still be busy, and leave the answer here)
        same = self._same_stream
        if same is None:
            same = self._torch.cuda.current_stream(self.device).cuda_stream == (stream or 0)
        if not same:
            t.record_stream(self._stream)
        p = t.data_ptr()
        self._live[p] = t
        return p

    def set_stream(self, stream):
        """Queue later calls on `stream` (a torch.cuda.Stream); they wait for
        the handle's work already queued on the old stream."""
        _check(self._lib.msp_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))
        self._stream = stream

    def _free(self, ctx, ptr, stream):
        self._live.pop(ptr, None)

    def _begin(self):
        """Compare torch's current stream with the handle's once per call,
        before the call (while the GPU may still be busy); every allocation
        of the call uses the answer."""
        self._same_stream = (self._torch.cuda.current_stream(self.device).cuda_stream ==
                             (self._stream.cuda_stream or 0))

    def _end(self):
        self._same_stream = None

    def _empty(self, shape, dtype):
        """An output tensor the library writes on the handle's stream."""
        t = self._torch.empty(shape, dtype=dtype, device=f"cuda:{self.device}")
        if not self._same_stream:
            t.record_stream(self._stream)
        return t

    def _take_c(self, ptr, nnz, vdtype):
        """Column and value views of C's single allocation (values start at
        the next 256-byte boundary after the columns)."""
        t = self._live.pop(ptr)
        voff = (nnz * 4 + 255) & ~255
        vsz = self._torch.empty(0, dtype=vdtype).element_size()
        return t[: nnz * 4].view(self._torch.int32), t[voff: voff + nnz * vsz].view(vdtype)

    def close(self):
        if self._h:
            self._lib.msp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, on: bool = True, phases=None):
        """Enable (and reset) per-phase HIP-event timing: every phase, or only
        the named ones (names as in PHASES)."""
        mask = 0
        if on:
            mask = -1 if phases is None else sum(1 << PHASES.index(p) for p in phases)
        _check(self._lib.msp_profile_enable(self._h, mask))

    def profile_get(self) -> dict:
        """{phase: (total ms, intervals)} for every phase timed so far."""
        p = c_profile()
        _check(self._lib.msp_profile_get(self._h, ctypes.byref(p)))
        return {name: (p.ms[i], int(p.count[i])) for i, name in enumerate(PHASES)}

    def set_tuning(self, tuning):
        _check(self._lib.msp_set_tuning(self._h, ctypes.byref(c_tuning(*tuning))))

    def summary_fallbacks(self) -> int:
        """Times a pass summary was read from a device copy because the
        kernel's direct write to host memory had not yet arrived."""
        f = self._lib.msp_internal_summary_fallbacks
        f.argtypes = [ctypes.c_void_p]
        f.restype = ctypes.c_longlong
        return int(f(self._h))

    def get_tuning(self):
        t = c_tuning()
        _check(self._lib.msp_get_tuning(self._h, ctypes.byref(t)))
        return _tuple(t)

    def sync(self):
        """Wait for the handle's stream; raise on any internal error that the
        numeric kernels of earlier calls flagged."""
        _check(self._lib.msp_sync(self._h))

    def spgemm(self, A: DeviceCSR, B: DeviceCSR, validate=False, force_spill=False,
               tuning=None, row_ptr=None, check=True) -> DeviceCSR:
        """C = A * B (plain two-phase path).  With check, wait for the
        result and raise on internal errors (msp_sync)."""
        torch = self._torch
        a, b = A.c(), B.c()
        out = c_csr_out()
        self._begin()
        try:
            rp = row_ptr if row_ptr is not None else self._empty(A.nrows + 1, torch.int64)
            out.row_ptr = rp.data_ptr()
            o = _opts(validate, force_spill, tuning)
            _check(self._lib.msp_spgemm(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(out),
                                        ctypes.byref(o)))
        finally:
            self._end()
        nnz = int(out.nnz)
        vdt = torch.float64 if out.dtype == MSP_F64 else torch.float32
        if nnz > 0:
            col, val = self._take_c(out.col, nnz, vdt)
        else:
            col = torch.empty(0, dtype=torch.int32, device=rp.device)
            val = torch.empty(0, dtype=vdt, device=rp.device)
        if check:
            self.sync()
        return DeviceCSR(A.nrows, B.ncols, rp, col, val)

    def spgemm_learned(self, pred: "Predictor", A: DeviceCSR, B: DeviceCSR, validate=False,
                       force_spill=False, tuning=None, check=True):
        """C = A * B in one pass sized by the predictor; returns (C, stats)."""
        torch = self._torch
        a, b = A.c(), B.c()
        out = c_csr_out()
        self._begin()
        try:
            rp = self._empty(A.nrows + 1, torch.int64)
            out.row_ptr = rp.data_ptr()
            st = c_learned_stats()
            o = _opts(validate, force_spill, tuning)
            _check(self._lib.msp_spgemm_learned(self._h, pred._p, ctypes.byref(a), ctypes.byref(b),
                                                ctypes.byref(out), ctypes.byref(o), ctypes.byref(st)))
        finally:
            self._end()
        nnz = int(out.nnz)
        vdt = torch.float64 if out.dtype == MSP_F64 else torch.float32
        if nnz > 0:
            col, val = self._take_c(out.col, nnz, vdt)
        else:
            col = torch.empty(0, dtype=torch.int32, device=rp.device)
            val = torch.empty(0, dtype=vdt, device=rp.device)
        if check:
            self.sync()
        stats = {"overflow_rows": int(st.overflow_rows), "sum_cap": int(st.sum_cap), "nnz": int(st.nnz),
                 "exact_rows": int(st.exact_rows)}
        return DeviceCSR(A.nrows, B.ncols, rp, col, val), stats

    def training_rows(self, A: DeviceCSR, B: DeviceCSR, feats=None, targets=None):
        """(features m x 8, targets m) float32 for the rows of A*B; writes
        into the given tensors (views into a larger training set) if any."""
        torch = self._torch
        m = A.nrows
        self._begin()
        try:
            if feats is None:
                feats = self._empty((max(m, 1), 8), torch.float32)
            if targets is None:
                targets = self._empty(max(m, 1), torch.float32)
            a, b = A.c(), B.c()
            _check(self._lib.msp_training_rows(self._h, ctypes.byref(a), ctypes.byref(b),
                                               ctypes.c_void_p(feats.data_ptr()),
                                               ctypes.c_void_p(targets.data_ptr())))
        finally:
            self._end()
        return feats[:m], targets[:m]

    def symbolic(self, A: DeviceCSR, B: DeviceCSR, validate=False, force_spill=False, tuning=None):
        """(row_nnz int32 tensor, nnz(C)) from the symbolic pass alone."""
        torch = self._torch
        a, b = A.c(), B.c()
        self._begin()
        try:
            rn = self._empty(max(A.nrows, 1), torch.int32)
            tot = ctypes.c_int64()
            o = _opts(validate, force_spill, tuning)
            _check(self._lib.msp_spgemm_symbolic(self._h, ctypes.byref(a), ctypes.byref(b),
                                                 ctypes.c_void_p(rn.data_ptr()), ctypes.byref(tot),
                                                 ctypes.byref(o)))
        finally:
            self._end()
        return rn[: A.nrows], int(tot.value)

    def autotune(self, A: DeviceCSR, B: DeviceCSR, candidates, reps: int = 5):
        """Median time of whole msp_spgemm(A, B) calls under each candidate
        tuning; returns (best, times_ms).  The handle's tuning is unchanged."""
        n = len(candidates)
        arr = (c_tuning * n)(*[c_tuning(*t) for t in candidates])
        times = (ctypes.c_double * n)()
        best = c_tuning()
        a, b = A.c(), B.c()
        self._begin()
        try:
            _check(self._lib.msp_autotune(self._h, ctypes.byref(a), ctypes.byref(b), arr, n, reps,
                                          ctypes.byref(best), times))
        finally:
            self._end()
        times = [float(t) for t in times]
        return tuple(candidates[times.index(min(times))]), times

    def omar_distinct(self, A: DeviceCSR, group: int) -> int:
        """Distinct (row group, column) pairs of A for groups of `group`
        consecutive rows: the B-row reads of Eq. (1)'s buffering scheme."""
        out = ctypes.c_int64()
        a = A.c()
        _check(self._lib.msp_omar(self._h, ctypes.byref(a), int(group), ctypes.byref(out)))
        return int(out.value)

    def omar(self, A: DeviceCSR, group: int) -> float:
        """OMAR of Eq. (1) in percent."""
        return 100.0 * (A.nnz - self.omar_distinct(A, group)) / A.nnz if A.nnz else 0.0

    def share_stats(self) -> dict:
        """B-row sharing figures of the handle's last call (after a wait)."""
        st = c_share_stats()
        _check(self._lib.msp_share_stats_get(self._h, ctypes.byref(st)))
        return {"batches": st.batches, "a_entries": st.a_entries, "b_rows": st.b_rows}

    def row_features(self, A: DeviceCSR, B: DeviceCSR):
        """(prod int64 [m], features float32 [m, 8])."""
        torch = self._torch
        m = A.nrows
        self._begin()
        try:
            prod = self._empty(max(m, 1), torch.int64)
            feat = self._empty((max(m, 1), 8), torch.float32)
            a, b = A.c(), B.c()
            _check(self._lib.msp_row_features(self._h, ctypes.byref(a), ctypes.byref(b),
                                              ctypes.c_void_p(prod.data_ptr()),
                                              ctypes.c_void_p(feat.data_ptr())))
        finally:
            self._end()
        return prod[:m], feat[:m]


NPARAM = 4801
BLOB_BYTES = 57644          # MSP_PREDICTOR_BLOB_BYTES


def blob_pack(params, delta: float = 0.0, adam_m=None, adam_v=None, step: int = 0) -> bytes:
    """Host-only: the predictor blob of the given state (no device needed)."""
    lib = load()
    arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float32) for a in (params, adam_m, adam_v)]
    for a in arrs:
        assert a is None or a.size == NPARAM
    ptr = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)   # noqa: E731
    buf = ctypes.create_string_buffer(BLOB_BYTES)
    size = ctypes.c_size_t()
    _check(lib.msp_predictor_blob_pack(ptr(arrs[0]), ptr(arrs[1]), ptr(arrs[2]), ctypes.c_float(delta),
                                       ctypes.c_int64(step), buf, BLOB_BYTES, ctypes.byref(size)))
    return buf.raw[: size.value]


def blob_unpack(blob: bytes):
    """Host-only: (params, delta, adam_m, adam_v, step) from a blob."""
    lib = load()
    out = [np.zeros(NPARAM, dtype=np.float32) for _ in range(3)]
    d = ctypes.c_float()
    st = ctypes.c_int64()
    _check(lib.msp_predictor_blob_unpack(blob, len(blob), *[a.ctypes.data_as(ctypes.c_void_p) for a in out],
                                         ctypes.byref(d), ctypes.byref(st)))
    return out[0], float(d.value), out[1], out[2], int(st.value)


class Predictor:
    """The FP32 8-64-64-1 output-size network on the handle's device."""

    def __init__(self, handle: Handle, params):
        self.h = handle
        self._lib = handle._lib
        self._p = ctypes.c_void_p()
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == NPARAM
        _check(self._lib.msp_predictor_create(handle._h, p.ctypes.data_as(ctypes.c_void_p),
                                              ctypes.byref(self._p)))

    def close(self):
        if self._p:
            self._lib.msp_predictor_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get(self):
        out = np.zeros(NPARAM, dtype=np.float32)
        d = ctypes.c_float()
        _check(self._lib.msp_predictor_get(self.h._h, self._p, out.ctypes.data_as(ctypes.c_void_p),
                                           ctypes.byref(d)))
        return out, float(d.value)

    def set(self, params=None, delta: float = 0.0):
        ptr = None
        if params is not None:
            p = np.ascontiguousarray(params, dtype=np.float32)
            ptr = p.ctypes.data_as(ctypes.c_void_p)
        _check(self._lib.msp_predictor_set(self.h._h, self._p, ptr, ctypes.c_float(delta)))

    def save(self) -> bytes:
        """The predictor's state (parameters, delta, Adam moments and step
        count) as the versioned blob of msp_predictor_save."""
        buf = ctypes.create_string_buffer(BLOB_BYTES)
        size = ctypes.c_size_t()
        _check(self._lib.msp_predictor_save(self.h._h, self._p, buf, BLOB_BYTES, ctypes.byref(size)))
        return buf.raw[: size.value]

    def load(self, blob: bytes):
        """Replace the state from a blob written by save()."""
        _check(self._lib.msp_predictor_load(self.h._h, self._p, blob, len(blob)))

    def train(self, feats, targets, batch_idx, lr=1e-3):
        """feats (n x 8), targets (n) float32 and batch_idx (steps x batch)
        int32 device tensors; returns the per-step losses."""
        steps, batch = batch_idx.shape
        losses = np.zeros(max(steps, 1), dtype=np.float32)
        o = c_train_opts(lr, 0.0, 0.0, 0.0)
        _check(self._lib.msp_predictor_train(self.h._h, self._p, feats.data_ptr(), targets.data_ptr(),
                                             feats.shape[0], batch_idx.data_ptr(), steps, batch,
                                             ctypes.byref(o), losses.ctypes.data_as(ctypes.c_void_p)))
        return losses[:steps]

    def grad(self, feats, targets, idx):
        g = np.zeros(NPARAM, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        _check(self._lib.msp_predictor_grad(self.h._h, self._p, feats.data_ptr(), targets.data_ptr(),
                                            feats.shape[0], idx.data_ptr(), idx.numel(),
                                            g.ctypes.data_as(ctypes.c_void_p),
                                            loss.ctypes.data_as(ctypes.c_void_p)))
        return float(loss[0]), g

    def infer(self, feats):
        import torch
        self.h._begin()
        try:
            y = self.h._empty(max(feats.shape[0], 1), torch.float32)
            _check(self._lib.msp_predictor_infer(self.h._h, self._p, feats.data_ptr(), feats.shape[0],
                                                 y.data_ptr()))
        finally:
            self.h._end()
        return y[: feats.shape[0]]

    def calibrate(self, feats, targets, q=0.99):
        _check(self._lib.msp_predictor_calibrate(self.h._h, self._p, feats.data_ptr(), targets.data_ptr(),
                                                 feats.shape[0], ctypes.c_double(q)))
        return self.get()[1]


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------

@dataclass
class PackedBatch:
    """A batch in packed form (see msp_batch_csr): device row_ptr/col/val,
    host row_start (nprob + 1) and ncols (nprob)."""
    row_start: np.ndarray
    ncols: np.ndarray
    row_ptr: object
    col: object
    val: object

    @property
    def nprob(self) -> int:
        return int(self.ncols.size)

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @classmethod
    def from_host(cls, mats, device="cuda") -> "PackedBatch":
        """Pack host CSR matrices (gen.CSR) into one device batch."""
        import torch
        row_start = np.zeros(len(mats) + 1, dtype=np.int64)
        np.cumsum([m.nrows for m in mats], out=row_start[1:])
        ncols = np.array([m.ncols for m in mats], dtype=np.int64)
        nnz_off = np.zeros(len(mats) + 1, dtype=np.int64)
        np.cumsum([m.nnz for m in mats], out=nnz_off[1:])
        rp = np.empty(int(row_start[-1]) + 1, dtype=np.int64)
        for i, m in enumerate(mats):
            rp[row_start[i]:row_start[i + 1]] = m.row_ptr[:-1] + nnz_off[i]
        rp[-1] = nnz_off[-1]
        col = np.concatenate([m.col for m in mats]) if mats else np.zeros(0, np.int32)
        val = np.concatenate([m.val for m in mats]) if mats else np.zeros(0)
        d = torch.device(device)
        return cls(row_start, ncols, torch.from_numpy(rp).to(d), torch.from_numpy(col.astype(np.int32)).to(d),
                   torch.from_numpy(val).to(d))

    def view(self, p: int) -> DeviceCSR:
        """Problem p as a single-product operand (row_ptr not starting at 0)."""
        r0, r1 = int(self.row_start[p]), int(self.row_start[p + 1])
        return DeviceCSR(r1 - r0, int(self.ncols[p]), self.row_ptr[r0:r1 + 1], self.col, self.val)

    def c(self) -> c_batch_csr:
        self._rs = np.ascontiguousarray(self.row_start, dtype=np.int64)
        self._nc = np.ascontiguousarray(self.ncols, dtype=np.int64)
        dt = MSP_F64 if self.val.dtype == self._torch_f64() else MSP_F32
        return c_batch_csr(self.nprob, self._rs.ctypes.data, self._nc.ctypes.data, self.nnz,
                           self.row_ptr.data_ptr(), self.col.data_ptr() if self.nnz else None,
                           self.val.data_ptr() if self.nnz else None, dt)

    @staticmethod
    def _torch_f64():
        import torch
        return torch.float64


class Batch:
    """A planned batch C_p = A_p P_p, or C_p = R_p (A_p P_p) with R."""

    def __init__(self, handle: "Handle", A: PackedBatch, P: PackedBatch, R: PackedBatch | None = None,
                 tuning=None, queue_rows: int = 0):
        """queue_rows: rows per ticket of the numeric merge's shared work
        queue (0: the library's 1024; -1: one static row range per wave)."""
        self.h = handle
        self._lib = handle._lib
        self._inputs = (A, P, R)                # the plan reads them on every replay
        ca, cp = A.c(), P.c()
        cr = R.c() if R is not None else None
        self._c = (ca, cp, cr)
        o = _opts(False, False, tuning, queue_rows)
        self._b = ctypes.c_void_p()
        _check(self._lib.msp_batch_create(handle._h, ctypes.byref(cr) if cr is not None else None,
                                          ctypes.byref(ca), ctypes.byref(cp), ctypes.byref(o),
                                          ctypes.byref(self._b)))
        self.nprob = A.nprob

    def close(self):
        if self._b:
            self._lib.msp_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def execute(self):
        _check(self._lib.msp_batch_execute(self.h._h, self._b))

    def sync(self):
        _check(self._lib.msp_batch_sync(self.h._h, self._b))

    def result(self, p: int) -> DeviceCSR:
        """Problem p of the last replay, copied out of the plan's arena."""
        torch = self.h._torch
        out = c_csr_out()
        _check(self._lib.msp_batch_copy_result(self.h._h, self._b, p, ctypes.byref(out)))
        rp = self.h._live.pop(out.row_ptr)[: (out.nrows + 1) * 8].view(torch.int64)
        nnz = int(out.nnz)
        vdt = torch.float64 if out.dtype == MSP_F64 else torch.float32
        if nnz > 0:
            col, val = self.h._take_c(out.col, nnz, vdt)
        else:
            col = torch.empty(0, dtype=torch.int32, device=rp.device)
            val = torch.empty(0, dtype=vdt, device=rp.device)
        return DeviceCSR(int(out.nrows), int(out.ncols), rp, col, val)

    def info(self) -> dict:
        st = c_batch_stats()
        _check(self._lib.msp_batch_info(self._b, ctypes.byref(st)))
        n = st.nstage
        return {"nstage": n, "rows": list(st.rows)[:n], "nnz": list(st.nnz)[:n],
                "sym_bins": list(st.sym_bins)[:n], "num_bins": list(st.num_bins)[:n]}


def autotune(handle: "Handle", A: PackedBatch, P: PackedBatch, R: PackedBatch | None, candidates, reps=5):
    """Median replay time of each candidate tuning; returns (best, times_ms)."""
    n = len(candidates)
    arr = (c_tuning * n)(*[c_tuning(*t) for t in candidates])
    times = (ctypes.c_double * n)()
    best = c_tuning()
    ca, cp = A.c(), P.c()
    cr = R.c() if R is not None else None
    _check(handle._lib.msp_batch_autotune(handle._h, ctypes.byref(cr) if cr is not None else None,
                                          ctypes.byref(ca), ctypes.byref(cp), arr, n, reps,
                                          ctypes.byref(best), times))
    times = [float(t) for t in times]
    return tuple(candidates[times.index(min(times))]), times


def tuning_to_json(t) -> str:
    lib = load()
    ct = c_tuning(*t)
    n = lib.msp_tuning_to_json(ctypes.byref(ct), None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    lib.msp_tuning_to_json(ctypes.byref(ct), buf, n + 1)
    return buf.value.decode()


def tuning_from_json(js: str):
    lib = load()
    ct = c_tuning()
    _check(lib.msp_tuning_from_json(js.encode(), ctypes.byref(ct)))
    return _tuple(ct)
