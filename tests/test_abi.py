"""CPU-side checks of the C ABI: the library loads, exports every declared entry point, and
rejects invalid arguments before touching the device."""
import ctypes
import re

import pytest


@pytest.fixture(scope="module")
def L():
    from paper_1205_2288_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol(L):
    declared = L.header_symbols()
    assert len(declared) >= 19
    for name in declared:
        assert hasattr(L.lib, name), name


def test_version_and_status_strings(L):
    assert L.tsbts_version() >= 10000
    for st in (L.TSBTS_OK, L.TSBTS_EINVAL, L.TSBTS_ENOMEM, L.TSBTS_EHIP, L.TSBTS_ESTATE):
        assert L.tsbts_strerror(st) and L.tsbts_strerror(st) != "unknown status"


def test_create_rejects_bad_arguments_without_a_device(L):
    out = ctypes.c_void_p()
    assert L.lib.tsbts_create(None, 10, 0.1, L.TSBTS_MIXED, 0) == L.TSBTS_EINVAL
    assert L.lib.tsbts_create(ctypes.byref(out), 0, 0.1, L.TSBTS_MIXED, 0) == L.TSBTS_EINVAL
    assert L.lib.tsbts_create(ctypes.byref(out), 10, -1.0, L.TSBTS_MIXED, 0) == L.TSBTS_EINVAL
    assert L.lib.tsbts_create(ctypes.byref(out), 10, float("nan"), 0, 0) == L.TSBTS_EINVAL
    assert L.lib.tsbts_create(ctypes.byref(out), 10, 0.1, 7, 0) == L.TSBTS_EINVAL
    assert L.lib.tsbts_create(ctypes.byref(out), 10, 0.1, 0, 64) == L.TSBTS_EINVAL
    assert out.value is None


def test_null_context_is_rejected(L):
    assert L.lib.tsbts_predict(None, 0.0, 0, None) == L.TSBTS_EINVAL
    assert L.lib.tsbts_force(None, None, 1, 0.0, None, None, None) == L.TSBTS_EINVAL
    assert L.lib.tsbts_destroy(None) == L.TSBTS_OK


def test_header_documents_each_entry_point():
    import os
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "tsbts.h")).read()
    # every declaration is preceded by a comment block
    for m in re.finditer(r"\n(int|const char \*)\s*(tsbts_[a-z_]+)\(", hdr):
        before = hdr[:m.start()].rstrip()
        assert before.endswith("*/"), m.group(2)
