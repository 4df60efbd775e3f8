"""The C ABI library loads on the CPU and exports every symbol include/ivx.h declares;
host-side argument validation works without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ivx.h")
LIB = os.path.join(ROOT, "paper_1906_08556_amd", "libivx.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    # function-pointer typedefs (callback types) declare no symbol
    src = re.sub(r"typedef\s+\w+\s*\(\s*\*\s*\w+\s*\)\s*\([^)]*\)\s*;", "", src)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ["ubm_posteriors", "bw_stats", "tv_estep", "tv_mstep_accumulate", "extract_ivectors",
              "tv_mstep_solve", "tv_mindiv", "ubm_update_means", "ivx_create", "ivx_destroy",
              "ivx_set_ubm", "ivx_init_tv", "ivx_set_tv", "ivx_get_tv", "ivx_sync_status",
              "ivx_last_error", "ivx_tp_size"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libivx.so not built")
    lib = ctypes.CDLL(LIB)
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_prototypes_cover_the_header():
    from paper_1906_08556_amd import ivx
    assert sorted(ivx.PROTOTYPES) == _declared()


def test_host_validation_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("libivx.so not built")
    from paper_1906_08556_amd import ivx
    lib = ivx.load()
    h = ctypes.c_void_p()
    bad = ivx.Dims(0, 60, 400, 10, 1000)
    assert lib.ivx_create(ctypes.byref(bad), 0, ctypes.byref(h)) == -1
    assert b"C=0" in lib.ivx_last_error()
    bad = ivx.Dims(16, 64, 400, 10, 1000)
    assert lib.ivx_create(ctypes.byref(bad), 0, ctypes.byref(h)) == -1
    # slot ids (frame * 32 proposal slots) must fit in int32: 2^26 frames is
    # the first batch size refused, 2^26 - 1 the last accepted by the check
    big = ivx.Dims(16, 20, 32, 10, 1 << 26)
    assert lib.ivx_create(ctypes.byref(big), 0, ctypes.byref(h)) == -1
    assert b"max_batch_frames=67108864 out of range [1, 67108863]" in lib.ivx_last_error()
    # null context is rejected before any HIP call
    assert lib.ubm_posteriors(None, None, 0, 0, 0, None, None, None, 8, None, None) == -1
    assert lib.bw_stats(None, None, None, 1, 0, 0, 0, None, None, None, None, None) == -1
    assert lib.ivx_tp_size(400) == 25 * 26 // 2 * 256
    assert lib.ivx_tp_size(20) == 3 * 256
