"""The C-ABI library loads and exports every entry point include/hme.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

import paper_2507_21039_amd as hme

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "hme.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hme_[a-z_]+)\s*\(", src)))


def test_header_declares_expected_entry_points():
    assert set(hme.EXPORTED) <= set(declared_symbols())


@pytest.mark.skipif(not os.path.exists(hme.LIB_PATH), reason="libhme.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(hme.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(L, name), name


@pytest.mark.skipif(not os.path.exists(hme.LIB_PATH), reason="libhme.so not built")
def test_argument_errors_without_gpu():
    # argument checks happen before any device call
    L = hme.lib()
    h = ctypes.c_void_p()
    assert L.hme_create(0, None, 0, 0, ctypes.byref(h)) == hme.HME_E_ARG
    assert "card" in hme.last_error()
    card = hme.card_struct((91.188, 2.441, 132.5, 1.16639e-5, 173.0, 0.0))
    assert L.hme_create(99, ctypes.byref(card), 0, 0, ctypes.byref(h)) == hme.HME_E_ARG
    assert L.hme_create(0, ctypes.byref(card), 7, 0, ctypes.byref(h)) == hme.HME_E_ARG
    assert L.hme_compute(None, 0.118, 10, None, None, None) == hme.HME_E_ARG
    assert L.hme_destroy(None) == hme.HME_OK
    info = hme.Info()
    assert L.hme_query(None, ctypes.byref(info)) == hme.HME_E_ARG


@pytest.mark.skipif(not os.path.exists(hme.LIB_PATH), reason="libhme.so not built")
def test_phase_space_argument_errors_without_gpu():
    L = hme.lib()
    card = hme.card_struct((91.188, 2.441, 132.5, 1.16639e-5, 173.0, 0.0))
    buf = ctypes.c_void_p(8)  # never dereferenced: every call below fails its checks first
    assert L.hme_rambo(9, ctypes.byref(card), 1000.0, 1, 0, 10, 0, 0.0, buf, None, None) == hme.HME_E_ARG
    assert L.hme_rambo(1, None, 1000.0, 1, 0, 10, 0, 0.0, buf, None, None) == hme.HME_E_ARG
    assert L.hme_rambo(1, ctypes.byref(card), 1000.0, 1, 0, -1, 0, 0.0, buf, None, None) == hme.HME_E_ARG
    assert L.hme_rambo(1, ctypes.byref(card), 1000.0, 1, 0, 10, 3, 0.0, buf, None, None) == hme.HME_E_ARG
    assert "cut" in hme.last_error()
    assert L.hme_rambo(1, ctypes.byref(card), 300.0, 1, 0, 10, 0, 0.0, buf, None, None) == hme.HME_E_ARG
    assert "sqrt_s" in hme.last_error()
    assert L.hme_rambo(1, ctypes.byref(card), 1000.0, 1, 0, 10, 0, 0.0, None, None, None) == hme.HME_E_ARG
    assert L.hme_rambo(1, ctypes.byref(card), 1000.0, 1, 0, 10, 0, 0.0, ctypes.c_void_p(12), None,
                       None) == hme.HME_E_ARG
    # e+e- -> mu+mu- has massless final states: any positive energy is above threshold
    assert L.hme_rambo(0, ctypes.byref(card), 100.0, 1, 0, 0, 0, 0.0, None, None, None) == hme.HME_OK
    assert L.hme_weighted_sum(buf, buf, -1, buf, None) == hme.HME_E_ARG
    assert L.hme_weighted_sum(buf, buf, 10, None, None) == hme.HME_E_ARG
    assert L.hme_weighted_sum(None, buf, 10, buf, None) == hme.HME_E_ARG


@pytest.mark.skipif(not os.path.exists(hme.LIB_PATH), reason="libhme.so not built")
def test_alphas_and_select_argument_errors_without_gpu():
    L = hme.lib()
    buf = ctypes.c_void_p(8)
    assert L.hme_compute_alphas(None, buf, 10, buf, buf, None) == hme.HME_E_ARG
    assert L.hme_compute_select(None, 0.118, 10, buf, buf, buf, buf, buf, buf, None) == hme.HME_E_ARG
