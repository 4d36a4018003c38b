"""The C-ABI library loads on the CPU, exports every symbol include/msp.h
declares, and rejects bad arguments on the host (no GPU calls)."""
import ctypes
import os
import re

import pytest

from paper_2112_10037_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "msp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(msp_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = _declared()
    assert "msp_spgemm" in names and len(names) >= 10
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/msp.h but not exported"
    bound = {s[0] for s in binding.SIGNATURES}
    assert set(names) <= bound, f"binding lacks {set(names) - bound}"


def test_every_tuning_plan_has_a_kernel():
    lib = ctypes.CDLL(binding.LIB_PATH)
    lib.msp_internal_unsupported_plans.argtypes = [ctypes.c_int]
    assert lib.msp_internal_unsupported_plans(0) == 0


def test_status_strings_and_null_handle():
    lib = binding.load()
    for code in range(9):
        assert lib.msp_status_string(code)
    # NULL handle: rejected on the host before any device call
    assert lib.msp_spgemm(None, None, None, None, None) == 1
    assert b"null handle" in lib.msp_last_error()
    assert lib.msp_destroy(None) == 0
    assert lib.msp_set_tuning(None, None) == 1


def test_tuning_json_roundtrip_and_rejects():
    from paper_2112_10037_amd import binding
    for t in [(1, 0, 4096, 128, 8), (2, 2, 256, 32, -1), (1, 1, 1024, 64, 4)]:
        js = binding.tuning_to_json(t)
        assert binding.tuning_from_json(js) == t
    # field order and spacing are free
    assert binding.tuning_from_json('{"merge_k":4,"block_rows":64,"spill_nnz":512,'
                                    '"group_scale":1,"hash_scale":2}') == (2, 1, 512, 64, 4)
    import pytest
    with pytest.raises(binding.MspError):
        binding.tuning_from_json('{"hash_scale": 1}')
    with pytest.raises(binding.MspError):
        binding.tuning_from_json('{"hash_scale": 9, "group_scale": 0, "spill_nnz": 4096, '
                                 '"block_rows": 128, "merge_k": 8}')


def test_predictor_blob_roundtrip_and_rejects():
    """The versioned predictor blob (host arrays only): a round trip keeps
    every byte of the state; a wrong magic, version, count, size or hash
    is refused."""
    import struct

    import numpy as np
    rng = np.random.default_rng(3)
    p, m, v = (rng.standard_normal(binding.NPARAM).astype(np.float32) for _ in range(3))
    blob = binding.blob_pack(p, 0.625, m, v, 1234)
    assert len(blob) == binding.BLOB_BYTES == 24 + 3 * 4 * binding.NPARAM + 8
    assert blob[:4] == b"MSPP" and struct.unpack_from("<IIfq", blob, 4) == (1, binding.NPARAM, 0.625, 1234)
    q, d, qm, qv, st = binding.blob_unpack(blob)
    assert np.array_equal(q, p) and np.array_equal(qm, m) and np.array_equal(qv, v)
    assert d == 0.625 and st == 1234
    # the parameters sit right after the header, in creation order
    assert np.array_equal(np.frombuffer(blob, np.float32, binding.NPARAM, 24), p)
    # missing moments pack as zeros
    _, _, zm, zv, _ = binding.blob_unpack(binding.blob_pack(p))
    assert not zm.any() and not zv.any()

    def refused(b, name):
        with pytest.raises(binding.MspError) as e:
            binding.blob_unpack(b)
        assert e.value.name == name

    refused(b"XSPP" + blob[4:], "MSP_ERR_INVALID_ARG")
    refused(blob[:4] + struct.pack("<I", 2) + blob[8:], "MSP_ERR_UNSUPPORTED")
    refused(blob[:8] + struct.pack("<I", 4800) + blob[12:], "MSP_ERR_INVALID_ARG")
    refused(blob[:-1], "MSP_ERR_INVALID_ARG")
    flipped = bytearray(blob)
    flipped[100] ^= 1                       # one parameter bit: the hash no longer matches
    refused(bytes(flipped), "MSP_ERR_INVALID_ARG")
    lib = binding.load()
    # size query, and a buffer one byte short
    size = ctypes.c_size_t()
    assert lib.msp_predictor_blob_pack(p.ctypes.data_as(ctypes.c_void_p), None, None, ctypes.c_float(0),
                                       0, None, 0, ctypes.byref(size)) == 0 and size.value == binding.BLOB_BYTES
    buf = ctypes.create_string_buffer(binding.BLOB_BYTES)
    assert lib.msp_predictor_blob_pack(p.ctypes.data_as(ctypes.c_void_p), None, None, ctypes.c_float(0),
                                       0, buf, binding.BLOB_BYTES - 1, None) == 1


def test_autotune_rejects_bad_arguments_on_the_host():
    lib = binding.load()
    assert lib.msp_autotune(None, None, None, None, 0, 1, None, None) == 1
