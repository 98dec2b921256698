"""The C-ABI library loads on a machine without a GPU and exports every function that
include/eifp.h declares; the Python binding names each of them (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eifp.h")
LIB = os.path.join(ROOT, "paper_2210_06232_amd", "libeifp.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eifp_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("eifp_init", "eifp_step", "eifp_invariants", "eifp_fields", "eifp_destroy"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libeifp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libeifp.so not built")
def test_binding_covers_the_header_and_status_strings():
    from paper_2210_06232_amd import eifp
    assert set(declared_functions()) == set(eifp.SIGNATURES)
    lib = eifp.load()
    # pure host functions are safe without a device
    assert lib.eifp_status_string(0) == b"ok"
    assert lib.eifp_status_string(2) == b"unsupported grid size"
    assert lib.eifp_stream(None) is None
    assert lib.eifp_device_bytes(None) == 0
    assert lib.eifp_destroy(None) == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="libeifp.so not built")
def test_argument_validation_needs_no_device():
    # every check below fails before any HIP call is made
    import numpy as np
    from paper_2210_06232_amd import eifp
    H = np.zeros((3, 8, 8, 8))
    dom = (0, 1, 0, 1, 0, 1)
    cases = [
        ((7, 8, 8, dom, 1.0, 1.0), eifp.EIFP_ERR_INVALID_ARG),      # odd size
        ((2, 8, 8, dom, 1.0, 1.0), eifp.EIFP_ERR_INVALID_ARG),      # below 4
        ((10, 8, 8, dom, 1.0, 1.0), eifp.EIFP_ERR_UNSUPPORTED_SIZE),  # factor 5
        ((1024, 8, 8, dom, 1.0, 1.0), eifp.EIFP_ERR_UNSUPPORTED_SIZE),
        ((8, 8, 8, (0, 0, 0, 1, 0, 1), 1.0, 1.0), eifp.EIFP_ERR_INVALID_ARG),
        ((8, 8, 8, dom, -1.0, 1.0), eifp.EIFP_ERR_INVALID_ARG),
        ((8, 8, 8, dom, 1.0, float("nan")), eifp.EIFP_ERR_INVALID_ARG),
    ]
    lib = eifp.load()
    for (nx, ny, nz, d, mu, eps), want in cases:
        Hc = np.zeros((3, nz, ny, nx))
        h = ctypes.c_void_p()
        st = lib.eifp_init(ctypes.byref(h), nx, ny, nz, ctypes.byref(eifp.eifp_domain(*d)), mu, eps, 0,
                           eifp._dp(Hc), eifp._dp(Hc), None)
        assert st == want, (nx, ny, nz, d, mu, eps, st)
        assert h.value is None
        assert lib.eifp_last_error()
    bad = H.copy()
    bad[1, 2, 3, 4] = np.inf
    h = ctypes.c_void_p()
    st = lib.eifp_init(ctypes.byref(h), 8, 8, 8, ctypes.byref(eifp.eifp_domain(*dom)), 1.0, 1.0, 0,
                       eifp._dp(bad), eifp._dp(H), None)
    assert st == eifp.EIFP_ERR_NONFINITE
    assert lib.eifp_step(None, 0.1, 1) == eifp.EIFP_ERR_INVALID_ARG
    assert lib.eifp_invariants(None, None) == eifp.EIFP_ERR_INVALID_ARG
