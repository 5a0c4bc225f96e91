"""The C-ABI library loads and exports every function include/sht.h declares;
the host-side argument checks reject bad plans before any device work.  No
compute call is made here (these run without a GPU)."""

import ctypes
import os
import re

import pytest

from paper_1908_06096_amd import sht

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sht.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sht_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("sht_plan_create", "sht_plan_destroy", "sht_inverse", "sht_direct", "sht_workspace_size"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = sht.library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_exactly_the_header():
    assert sht.exported_symbols() == _declared()


def test_strerror_texts():
    lib = sht.library()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.sht_strerror(code)
    assert b"unknown" in lib.sht_strerror(-99)


@pytest.mark.parametrize("args,code", [
    ((0, 0, 1, 0), -1),     # truncation 0
    ((79, 0, 0, 0), -1),    # no fields
    ((79, 5, 1, 0), -1),    # bad grid
    ((79, 0, 1, 9), -1),    # bad precision
    ((80, 0, 1, 0), -2),    # full grid with even N has an unpaired equator ring
])
def test_plan_create_rejects_bad_arguments_on_host(args, code):
    lib = sht.library()
    h = ctypes.c_void_p()
    assert lib.sht_plan_create(ctypes.byref(h), *args, None) == code
    assert not h.value


def test_null_handles_rejected():
    lib = sht.library()
    assert lib.sht_plan_create(None, 79, 0, 1, 0, None) == -1
    assert lib.sht_plan_destroy(None) == -1
    assert lib.sht_inverse(None, None, None, None, None) == -1
    assert lib.sht_direct(None, None, None, None, None) == -1
    assert lib.sht_workspace_size(None) == 0
    assert lib.sht_transform_static(None, 0, None, None, None) == -1
    assert lib.sht_stepper_create(None, None, 0.1, 1.0, 0.0, None, None, None, 0, 1, None) == -1
    assert lib.sht_stepper_run(None, 1, None) == -1
    assert lib.sht_stepper_destroy(None) == -1
    assert lib.sht_vector_inverse(None, None, None, None, None) == -1
    assert lib.sht_vector_direct(None, None, None, None, None) == -1
    assert lib.sht_gradient(None, None, None, None, None) == -1
    assert lib.sht_spectral_op(None, 0, 1, None, None, None) == -1
