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
