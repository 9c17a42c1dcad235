"""The C-ABI library loads, exports every symbol include/soft.h declares, and
rejects bad arguments before touching a GPU (CPU-only checks)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "soft.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(soft_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_1808_00896_amd import soft
    return soft.lib()


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("soft_plan", "soft_forward", "soft_inverse", "soft_adjoint", "soft_adjoint_inverse",
              "soft_plan_destroy", "soft_plan_sizes", "soft_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings(L):
    from paper_1808_00896_amd import soft
    assert soft.status_string(0) == "ok"
    assert "invalid" in soft.status_string(-1)
    assert "unsupported" in soft.status_string(-2)
    assert soft.status_string(12345) == "unknown status"


def test_argument_errors_need_no_gpu(L):
    from paper_1808_00896_amd import soft
    h = ctypes.c_void_p()
    assert L.soft_plan(0, 1, 0, 0, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_plan(8, 0, 0, 0, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_plan(8, 1, 0, 32, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    # the double-double recurrence is an FP64 option
    assert L.soft_plan(8, 1, soft.SOFT_FP32, soft.SOFT_DD_RECURRENCE, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_plan(8, 1, soft.SOFT_FP32_SPLIT, soft.SOFT_DD_RECURRENCE, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_plan(8, 1, 0, 0x80000000, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_plan_describe(None, None, 0) == soft.SOFT_ERR_INVALID
    assert L.soft_plan(8, 1, 7, 0, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_plan(8, 1, 0, 0, None) == soft.SOFT_ERR_INVALID
    assert L.soft_plan(6, 1, 0, 0, ctypes.byref(h)) == soft.SOFT_ERR_UNSUPPORTED
    assert L.soft_plan(2048, 1, 0, 0, ctypes.byref(h)) == soft.SOFT_ERR_UNSUPPORTED
    assert L.soft_plan(8, 65536, 0, 0, ctypes.byref(h)) == soft.SOFT_ERR_UNSUPPORTED
    assert L.soft_match_plan(8, 65536, 0, 0, ctypes.byref(h)) == soft.SOFT_ERR_UNSUPPORTED
    assert h.value is None
    for name in ("soft_forward", "soft_inverse", "soft_adjoint", "soft_adjoint_inverse"):
        assert getattr(L, name)(None, None, None, None) == soft.SOFT_ERR_INVALID
    assert L.soft_plan_sizes(None, None, None, None) == soft.SOFT_ERR_INVALID
    assert L.soft_plan_destroy(None) == soft.SOFT_OK


def test_uneven_argument_errors_need_no_gpu(L):
    from paper_1808_00896_amd import soft
    h = ctypes.c_void_p()
    arr = (ctypes.c_int * 3)(8, 16, 4)
    assert L.soft_plan_uneven(None, 3, 0, 0, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_plan_uneven(arr, 0, 0, 0, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_plan_uneven(arr, 3, 3, 0, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_plan_uneven(arr, 3, 0, 32, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_plan_uneven(arr, 3, 0, 0, None) == soft.SOFT_ERR_INVALID
    bad = (ctypes.c_int * 3)(8, 0, 4)
    assert L.soft_plan_uneven(bad, 3, 0, 0, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    odd = (ctypes.c_int * 3)(8, 12, 4)
    assert L.soft_plan_uneven(odd, 3, 1, 0, ctypes.byref(h)) == soft.SOFT_ERR_UNSUPPORTED
    big = (ctypes.c_int * 2)(8, 2048)
    assert L.soft_plan_uneven(big, 2, 2, 0, ctypes.byref(h)) == soft.SOFT_ERR_UNSUPPORTED
    assert h.value is None
    assert L.soft_plan_offsets(None, None, None) == soft.SOFT_ERR_INVALID
    for prec in (soft.SOFT_FP32, soft.SOFT_FP32_SPLIT):
        assert L.soft_plan(8, 0, prec, 0, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
        assert L.soft_plan(12, 1, prec, 0, ctypes.byref(h)) == soft.SOFT_ERR_UNSUPPORTED


def test_match_argument_errors_need_no_gpu(L):
    from paper_1808_00896_amd import soft
    h = ctypes.c_void_p()
    assert L.soft_match_plan(0, 4, 0, 0, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_match_plan(8, 0, 0, 0, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_match_plan(8, 4, 5, 0, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_match_plan(8, 4, 0, 32, ctypes.byref(h)) == soft.SOFT_ERR_INVALID
    assert L.soft_match_plan(8, 4, 0, 0, None) == soft.SOFT_ERR_INVALID
    assert L.soft_match_plan(24, 4, 2, 0, ctypes.byref(h)) == soft.SOFT_ERR_UNSUPPORTED
    assert h.value is None
    assert L.soft_match(None, None, None, None, None, None) == soft.SOFT_ERR_INVALID
    assert L.soft_match_coeffs(None, None, None, None, None) == soft.SOFT_ERR_INVALID
    assert L.soft_match_coeffs_vjp(None, None, None, None, None, None, None) == soft.SOFT_ERR_INVALID
    assert L.soft_match_argmax(None, None, None, None) == soft.SOFT_ERR_INVALID
    assert L.soft_match_refine(None, None, None, None, None) == soft.SOFT_ERR_INVALID
    assert L.soft_sh_forward(0, 1, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == soft.SOFT_ERR_INVALID
    assert L.soft_sh_forward(8, 1, 0, None, ctypes.c_void_p(16), None) == soft.SOFT_ERR_INVALID
    assert L.soft_sh_forward(12, 1, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == soft.SOFT_ERR_UNSUPPORTED
    one = ctypes.c_void_p(16)  # never dereferenced: the arguments are rejected first
    assert L.soft_match_argmax_noalloc(8, 2, 0, None, one, None) == soft.SOFT_ERR_INVALID
    assert L.soft_match_argmax_noalloc(8, 2, 0, one, None, None) == soft.SOFT_ERR_INVALID
    assert L.soft_match_argmax_noalloc(0, 2, 0, one, one, None) == soft.SOFT_ERR_INVALID
    assert L.soft_match_argmax_noalloc(8, 0, 0, one, one, None) == soft.SOFT_ERR_INVALID
    assert L.soft_match_argmax_noalloc(8, 2, 3, one, one, None) == soft.SOFT_ERR_INVALID
    assert L.soft_match_argmax_noalloc(12, 2, 0, one, one, None) == soft.SOFT_ERR_UNSUPPORTED
    assert L.soft_match_argmax_noalloc(1024, 2, 0, one, one, None) == soft.SOFT_ERR_UNSUPPORTED
    assert L.soft_match_argmax_noalloc(8, 65536, 0, one, one, None) == soft.SOFT_ERR_UNSUPPORTED
    assert L.soft_match_sizes(None, None, None, None) == soft.SOFT_ERR_INVALID
    assert L.soft_match_plan_soft(None, None) == soft.SOFT_ERR_INVALID
    assert L.soft_match_destroy(None) == soft.SOFT_OK


def test_probe_argument_errors_need_no_gpu(L):
    from paper_1808_00896_amd import soft
    one = ctypes.c_void_p(16)  # never dereferenced: the arguments are rejected first
    assert L.soft_probe_copy(None, one, 16, None) == soft.SOFT_ERR_INVALID
    assert L.soft_probe_copy(one, one, 0, None) == soft.SOFT_ERR_INVALID
    assert L.soft_probe_copy(one, one, 24, None) == soft.SOFT_ERR_INVALID
    assert L.soft_probe_flops(3, 1, 1, one, None) == soft.SOFT_ERR_INVALID
    assert L.soft_probe_flops(0, 0, 1, one, None) == soft.SOFT_ERR_INVALID
    assert L.soft_probe_flops(1, 1, 1, None, None) == soft.SOFT_ERR_INVALID
    # flops per launch: 8 FMAs x 64 lanes x 2 (vector), 8 MFMAs x 2*16*16*4 (matrix), 4 waves a block
    assert L.soft_probe_flop_count(0, 3, 5) == 8 * 64 * 2 * 4 * 3 * 5
    assert L.soft_probe_flop_count(1, 3, 5) == 8 * 2048 * 4 * 3 * 5
    assert L.soft_probe_flop_count(2, 1, 1) == 8 * 2048 * 4
    assert L.soft_probe_flop_count(5, 1, 1) == 0.0


def test_flag_constants_match_header():
    """The binding's flag values are the header's."""
    import re
    from paper_1808_00896_amd import soft
    text = open(os.path.join(ROOT, "include", "soft.h")).read()
    vals = dict((k, int(v)) for k, v in
                re.findall(r"\b(SOFT_PLAN_TUNE|SOFT_INPLACE_OK|SOFT_PLAN_GRAPH)\s*=\s*(\d+)u", text))
    assert vals == {"SOFT_PLAN_TUNE": soft.SOFT_PLAN_TUNE, "SOFT_INPLACE_OK": soft.SOFT_INPLACE_OK,
                    "SOFT_PLAN_GRAPH": soft.SOFT_PLAN_GRAPH}
