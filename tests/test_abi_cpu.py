"""The C ABI library loads and exports what include/qms.h declares; argument
errors that are decided before any device call return their codes.  No
sorting work is launched here (no GPU in this environment)."""
import ctypes
import os
import re

import pytest

from paper_1804_10062_amd import qms

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "qms.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qms_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(qms.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = qms.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_tiles():
    t = qms.qms_get_tiles()
    assert t["base_tile"] % t["merge_tile"] == 0
    assert t["base_tile"] & (t["base_tile"] - 1) == 0


def test_argument_errors_before_device_work():
    lib = qms.load_library()
    assert lib.qms_sort(None, 0, qms.QMS_U32, None) == qms.QMS_OK
    assert lib.qms_sort(None, 1, qms.QMS_F32, None) == qms.QMS_OK
    assert lib.qms_sort(None, 5, 7, None) == qms.QMS_ERR_UNSUPPORTED
    assert "dtype" in qms.last_error()
    assert lib.qms_sort(None, 5, qms.QMS_U32, None) == qms.QMS_ERR_INVALID
    assert lib.qms_sort_pairs(None, None, 5, qms.QMS_U32, None) == qms.QMS_ERR_INVALID
    assert lib.qms_sort(ctypes.c_void_p(0x1002), 5, qms.QMS_U32, None) == qms.QMS_ERR_ALIGN
    assert lib.qms_sort(ctypes.c_void_p(0x1000), (1 << 32) + (1 << 25) + 1, qms.QMS_U32,
                            None) == qms.QMS_ERR_UNSUPPORTED
    assert lib.qms_sort_batch(None, None, None, None, 0, qms.QMS_U32, None) == qms.QMS_OK
    assert lib.qms_sort_batch(None, None, None, None, 3, qms.QMS_U32, None) == qms.QMS_ERR_INVALID


def test_binding_fails_loudly_without_library(tmp_path):
    saved = qms._lib
    try:
        qms._lib = None
        with pytest.raises(RuntimeError, match="not been built"):
            qms.load_library(str(tmp_path / "libqms.so"))
    finally:
        qms._lib = saved
