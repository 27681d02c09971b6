"""The C-ABI library loads and exports every function include/mcmp2.h
declares (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mcmp2.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mcmp2_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    from paper_2203_05632_amd._lib import EXPORTS
    assert sorted(EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    from paper_2203_05632_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmcmp2.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_last_error_is_callable_without_device():
    from paper_2203_05632_amd import load
    assert isinstance(load().mcmp2_last_error(), bytes)


def test_init_rejects_bad_arguments_before_touching_device():
    from paper_2203_05632_amd import load
    lib = load()
    out = ctypes.c_void_p()
    rc = lib.mcmp2_init(None, None, None, 1, 1, 2, 1, 0, 0, None, ctypes.byref(out))
    assert rc == -1 and b"null" in lib.mcmp2_last_error()


def test_set_interaction_rejects_null_context():
    from paper_2203_05632_amd import load
    lib = load()
    assert lib.mcmp2_set_interaction(None, 2) == -1 and b"null" in lib.mcmp2_last_error()


def test_step_accumulate_validates_before_touching_device():
    from paper_2203_05632_amd import load
    lib = load()
    p16 = ctypes.c_void_p(16)
    assert lib.mcmp2_step_accumulate(None, p16, p16, 1, p16, None, p16, p16, p16) == -1
    assert b"null accumulator" in lib.mcmp2_last_error()
    assert lib.mcmp2_step_accumulate(None, p16, p16, 1, p16, p16, p16, ctypes.c_void_p(24), p16) == -1
    assert b"16-byte aligned" in lib.mcmp2_last_error()
    assert lib.mcmp2_step_accumulate(None, p16, p16, 1, p16, p16, p16, p16, p16) == -1
    assert b"null argument" in lib.mcmp2_last_error()


def test_headline_traffic_record_matches_sources():
    """bench.py reports roofline.traffic from the counter record under
    profiles/ only while the SHA-256 of the kernel's sources matches it; a
    change to those sources must come with a re-taken record."""
    import bench
    assert bench.recorded_traffic("adj_gemm", "C4", "fp64") is not None
