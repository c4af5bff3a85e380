"""CPU-side checks of the C ABI: the library loads, exports every entry
point that include/msm.h declares, and rejects NULL contexts without
touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(msm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_path():
    names = declared_functions()
    for want in ("msm_project", "msm_enumerate_pairs", "msm_verify", "msm_create", "msm_destroy"):
        assert want in names


def test_library_exports_every_declared_symbol(msm):
    lib = ctypes.CDLL(msm.LIB_PATH)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing
    assert set(msm.EXPORTS) == set(declared_functions())


def test_version(msm):
    assert msm.msm_version() >= 100


def test_null_context_is_rejected(msm):
    L = msm.lib()
    m = ctypes.c_int64(7)
    assert L.msm_project(None, None, 0, 1, 1, None, 8, None, None) == msm.MSM_E_INVALID
    assert L.msm_enumerate_pairs(None, None, 0, 8, 4, 1, None, 0, ctypes.byref(m), None) == msm.MSM_E_INVALID
    assert L.msm_verify(None, None, 0, 1, 1, None, 0, 0, 0.5, None, 0, ctypes.byref(m), None) == msm.MSM_E_INVALID
    assert b"NULL" in L.msm_last_error(None)
    L.msm_destroy(None)


def test_create_without_device_fails_cleanly(msm):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    st = msm.lib().msm_create(0, ctypes.byref(h))
    assert st in (msm.MSM_E_INVALID, msm.MSM_E_HIP)
    assert not h.value
    assert msm.lib().msm_last_error(None)


def test_enumerate_groupings_host_only():
    """The grouping plan is host logic: C(k, h) groupings, or fewer
    hierarchical ones on j blocks when j * floor(ell / k) >= log2(n) + 8
    (15 for ell = 128, k = 8, h = 4, j = 2; 10 for ell = 60, k = 6, h = 2,
    j = 3; counted by enumerating every difference set by hand)."""
    from paper_0904_3151_amd import msm
    assert msm.msm_enumerate_groupings(1_000_000, 128, 8, 4) == (15, 2)
    assert msm.msm_enumerate_groupings(20_000, 60, 6, 2) == (10, 3)
    assert msm.msm_enumerate_groupings(4_000_000, 240, 10, 8) == (45, 0)   # j = 2 needs 45 = C(10, 8)
    assert msm.msm_enumerate_groupings(200_000, 64, 5, 3) == (10, 0)
    assert msm.msm_enumerate_groupings(3000, 16, 16, 2) == (120, 0)        # blocks of one bit
    assert msm.msm_enumerate_groupings(10, 10, 3, 0) == (1, 0)             # h = 0
    with pytest.raises(msm.MSMError):
        msm.msm_enumerate_groupings(100, 64, 3, 3)
