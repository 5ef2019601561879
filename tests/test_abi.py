"""CPU-side checks of the C ABI: the library loads and exports every symbol
that include/d2.h declares; the binding's struct layouts match the header."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "d2.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(d2_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    from paper_1510_00012_amd import d2
    assert _declared() == sorted(d2.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_1510_00012_amd import d2
    if not os.path.exists(d2.LIB_PATH):
        pytest.skip("libd2.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(d2.LIB_PATH)
    missing = [s for s in _declared() if not hasattr(lib, s)]
    assert not missing, missing


def test_struct_layouts_match_header():
    from paper_1510_00012_amd import d2
    # d2_badmm_params: 2 doubles + 6 int32 = 40 bytes, no padding
    assert ctypes.sizeof(d2.BadmmParams) == 40
    assert ctypes.sizeof(d2.OtParams) == 24
    assert ctypes.sizeof(d2.BadmmStats) == 24
    assert ctypes.sizeof(d2.RoundInfo) == 40
    # d2_sg_params: 2 doubles + 4 int32; d2_sg_stats: 2 int32, int64,
    # 2 int32, double
    assert ctypes.sizeof(d2.SgParams) == 32
    assert ctypes.sizeof(d2.SgStats) == 32


def test_create_without_gpu_fails_cleanly():
    """No exception crosses the ABI: without a usable device d2_create
    returns D2_EDEVICE (on a GPU host it succeeds)."""
    from paper_1510_00012_amd import d2
    if not os.path.exists(d2.LIB_PATH):
        pytest.skip("libd2.so not built")
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    lib = d2.load_library()
    h = ctypes.c_void_p()
    st = lib.d2_create(ctypes.byref(h), 0, 0, None)
    assert st == d2.D2_EDEVICE and not h.value
