"""CPU-side checks of the C ABI: the library loads, exports every entry
point the header declares, and fails cleanly where no device is usable."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "modalproj.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(modal_[A-Za-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1503_08809_amd import modalproj
    if not os.path.exists(modalproj.LIB_PATH):
        from paper_1503_08809_amd import build
        build.build()
    return modalproj.lib()


def test_header_declares_the_stage_calls():
    names = _declared()
    for n in ["modal_create", "modal_destroy", "modal_gauss_legendre", "modal_legendre_table",
              "modal_sph_bessel_table", "modal_beta", "modal_S", "modal_gamma_from_S",
              "modal_gamma"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    from paper_1503_08809_amd import modalproj
    assert sorted(modalproj.exported_symbols()) == _declared()


def test_status_strings(lib):
    for s in range(7):
        assert lib.modal_status_str(s)
    assert lib.modal_status_str(99) == b"unknown status"


def test_null_arguments_are_rejected_without_a_device(lib):
    assert lib.modal_create(None, 0, None) == 1                      # INVALID_ARG
    assert lib.modal_gamma(None, None, None, 0, None) == 1
    assert b"NULL" in lib.modal_last_error(None)
    assert lib.modal_destroy(None) == 0


def test_create_without_device_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    st = lib.modal_create(ctypes.byref(h), 0, None)
    assert st == 4                                                   # MODAL_ERR_DEVICE
    assert h.value is None
