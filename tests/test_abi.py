"""Host-side checks of the C ABI (no GPU calls): the library loads and exports
every function include/fastmap_hip.h declares, and the binding declares the
same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastmap_hip.h")
LIB = os.path.join(ROOT, "paper_2505_04612_amd", "libfastmap_hip.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_four_core_calls():
    names = declared()
    for n in ("fm_build_pair_grams", "fm_epipolar_loss_grad", "fm_adam_step", "fm_reweight"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2505_04612_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()
    assert sorted(_lib._SIGNATURES) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_every_call_rejects_a_null_context_without_a_device():
    """Host-side validation comes first: with a NULL context every call that
    takes one returns FM_EINVAL and touches no device (this runs on the CPU)."""
    from paper_2505_04612_amd import _lib
    lib = ctypes.CDLL(LIB)
    no_ctx = {"fm_create", "fm_destroy", "fm_last_error", "fm_version", "fm_scene_destroy", "fm_scene_work_items"}
    for name in _lib.EXPORTS:
        if name in no_ctx:
            continue
        restype, argtypes = _lib._SIGNATURES[name]
        f = getattr(lib, name)
        f.restype, f.argtypes = restype, argtypes
        args = [0.0 if a in (ctypes.c_float, ctypes.c_double) else
                (None if a is ctypes.c_void_p or (isinstance(a, type) and issubclass(a, ctypes._Pointer)) else 0)
                for a in argtypes]
        assert f(*args) == _lib.FM_EINVAL, name
    f = lib.fm_scene_work_items
    f.restype, f.argtypes = ctypes.c_int64, [ctypes.c_void_p]
    assert f(None) == -1
