"""Thin ctypes binding of ``libeifp.so`` (declared in ``include/eifp.h``).

Only argument marshalling lives here: every step of the method runs in the library's
HIP kernels.  If the library has not been built, importing this module raises -- there
is no CPU fallback.

Field arrays are float64 numpy arrays ``[3, nz, ny, nx]`` (x fastest); a domain is
``(xl, xr, yl, yr, zl, zr)``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libeifp.so")

EIFP_OK = 0
EIFP_ERR_INVALID_ARG = 1
EIFP_ERR_UNSUPPORTED_SIZE = 2
EIFP_ERR_OUT_OF_MEMORY = 3
EIFP_ERR_DEVICE = 4
EIFP_ERR_NONFINITE = 5
EIFP_ERR_STATE = 6

EIFP_FP64 = 0
EIFP_FP32 = 1
PRECISIONS = {"fp64": EIFP_FP64, "fp32": EIFP_FP32}

PASS_NAMES = ("x_fwd", "z_fwd", "y_fused", "z_inv", "x_inv", "finalize")


class eifp_domain(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("xl", "xr", "yl", "yr", "zl", "zr")]


class eifp_invariant_set(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double),
        ("steps_done", ctypes.c_longlong),
        ("energy", ctypes.c_double),
        ("helicity", ctypes.c_double),
        ("momentum", ctypes.c_double * 3),
        ("div_h_l2", ctypes.c_double),
        ("div_e_l2", ctypes.c_double),
    ]


# every symbol the header declares, with (restype, argtypes)
_VP = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "eifp_init": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(eifp_domain), ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int, _DP, _DP, _VP]),
    "eifp_step": (ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_longlong]),
    "eifp_step_timed": (ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_longlong, _DP]),
    "eifp_invariants": (ctypes.c_int, [_VP, ctypes.POINTER(eifp_invariant_set)]),
    "eifp_fields": (ctypes.c_int, [_VP, _DP, _DP]),
    "eifp_fields_device": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int]),
    "eifp_spectrum": (ctypes.c_int, [_VP, _DP]),
    "eifp_sync": (ctypes.c_int, [_VP]),
    "eifp_stream": (_VP, [_VP]),
    "eifp_device_bytes": (ctypes.c_longlong, [_VP]),
    "eifp_destroy": (ctypes.c_int, [_VP]),
    "eifp_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "eifp_last_error": (ctypes.c_char_p, []),
}

_lib = None


def library_path() -> str:
    return _LIB_PATH


def load() -> ctypes.CDLL:
    """Load libeifp.so; raises if it is missing (build it with ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is not built; run __graft_entry__.build() first "
                              "(the EI-FP library has no CPU fallback)")
        # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7; loading it
        # first makes the library bind to that same runtime instead of a second copy.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class EifpError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        self.status = status
        msg = lib.eifp_status_string(status).decode()
        detail = lib.eifp_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}): {detail}")


def _check(status: int, where: str):
    if status != EIFP_OK:
        raise EifpError(status, where)


def _field(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.ndim != 4 or a.shape[0] != 3:
        raise ValueError("field arrays must be [3, nz, ny, nx]")
    if shape is not None and a.shape != shape:
        raise ValueError(f"field shape {a.shape} != {shape}")
    return a


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_DP)


# ----------------------------------------------------------------------------------
# same-named functions (raw handles)
# ----------------------------------------------------------------------------------

def eifp_init(nx, ny, nz, domain, mu, eps, prec, H0, E0, stream=None) -> int:
    """Returns the raw solver handle (an int)."""
    lib = load()
    H0 = _field(H0, (3, nz, ny, nx))
    E0 = _field(E0, (3, nz, ny, nx))
    dom = eifp_domain(*[float(v) for v in domain])
    h = _VP()
    p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    _check(lib.eifp_init(ctypes.byref(h), nx, ny, nz, ctypes.byref(dom), float(mu), float(eps), p,
                         _dp(H0), _dp(E0), stream), "eifp_init")
    return h.value


def eifp_step(handle, tau, nsteps=1):
    _check(load().eifp_step(handle, float(tau), int(nsteps)), "eifp_step")


def eifp_step_timed(handle, tau, nsteps=1) -> dict:
    out = np.zeros(6)
    _check(load().eifp_step_timed(handle, float(tau), int(nsteps), _dp(out)), "eifp_step_timed")
    return dict(zip(PASS_NAMES, out.tolist()))


def eifp_invariants(handle) -> dict:
    inv = eifp_invariant_set()
    _check(load().eifp_invariants(handle, ctypes.byref(inv)), "eifp_invariants")
    return {"t": inv.t, "steps_done": inv.steps_done, "energy": inv.energy, "helicity": inv.helicity,
            "momentum": list(inv.momentum), "div_h_l2": inv.div_h_l2, "div_e_l2": inv.div_e_l2}


def eifp_fields(handle, shape):
    """shape = (nx, ny, nz); returns (H, E) as float64 [3, nz, ny, nx]."""
    nx, ny, nz = shape
    H = np.empty((3, nz, ny, nx))
    E = np.empty((3, nz, ny, nx))
    _check(load().eifp_fields(handle, _dp(H), _dp(E)), "eifp_fields")
    return H, E


def eifp_fields_device(handle, H_ptr: int, E_ptr: int, prec):
    p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    _check(load().eifp_fields_device(handle, H_ptr, E_ptr, p), "eifp_fields_device")


def eifp_spectrum(handle, shape) -> np.ndarray:
    """Packed half spectrum, complex128 [6, nz, ny, nx/2]."""
    nx, ny, nz = shape
    out = np.empty((6, nz, ny, nx // 2, 2))
    _check(load().eifp_spectrum(handle, _dp(out)), "eifp_spectrum")
    return out[..., 0] + 1j * out[..., 1]


def eifp_sync(handle):
    _check(load().eifp_sync(handle), "eifp_sync")


def eifp_stream(handle) -> int:
    return load().eifp_stream(handle) or 0


def eifp_device_bytes(handle) -> int:
    return int(load().eifp_device_bytes(handle))


def eifp_destroy(handle):
    _check(load().eifp_destroy(handle), "eifp_destroy")


# ----------------------------------------------------------------------------------
# convenience wrapper
# ----------------------------------------------------------------------------------

class Solver:
    """Owns one library solver.  ``Solver(H0, E0, domain, mu, eps, prec="fp64")``."""

    def __init__(self, H0, E0, domain, mu=1.0, eps=1.0, prec="fp64", stream=None):
        H0 = _field(H0)
        _, nz, ny, nx = H0.shape
        self.shape = (nx, ny, nz)
        self.domain = tuple(float(v) for v in domain)
        self.mu, self.eps, self.prec = float(mu), float(eps), prec
        self.handle = eifp_init(nx, ny, nz, self.domain, mu, eps, prec, H0, E0, stream)

    def step(self, tau, nsteps=1):
        eifp_step(self.handle, tau, nsteps)
        return self

    def step_timed(self, tau, nsteps=1) -> dict:
        return eifp_step_timed(self.handle, tau, nsteps)

    def invariants(self) -> dict:
        return eifp_invariants(self.handle)

    def fields(self):
        return eifp_fields(self.handle, self.shape)

    def spectrum(self) -> np.ndarray:
        return eifp_spectrum(self.handle, self.shape)

    def sync(self):
        eifp_sync(self.handle)

    @property
    def stream(self) -> int:
        return eifp_stream(self.handle)

    def device_bytes(self) -> int:
        return eifp_device_bytes(self.handle)

    def close(self):
        if self.handle:
            eifp_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
