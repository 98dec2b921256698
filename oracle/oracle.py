"""ctypes binding of ``eifp_oracle.c`` -- TEST INFRASTRUCTURE, NOT PRODUCT CODE.

A plain FP64 CPU reference of the time-exponential-integrator Fourier pseudospectral
(EI-FP) scheme of Wang & Jiang (arXiv:2210.06232).  Every arithmetic step lives in the
C file; this module only marshals numpy arrays.  Only the tests, the smoke check and
the benchmark's CPU-baseline leg may use it.

Field arrays are float64 ``[3, nz, ny, nx]`` (x fastest, the vector ordering of Sec. 2.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eifp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NINV = 26
INV_NAMES = (
    ["E1", "E2"] + [f"E3_{k}" for k in "xyz"] + [f"E4_{k}" for k in "xyz"]
    + [f"E5_{k}" for k in "xyz"] + [f"E6_{k}" for k in "xyz"]
    + ["H1", "H2"] + [f"M1_{k}" for k in "xyz"] + [f"M2_{k}" for k in "xyz"]
    + ["divH_l2", "divE_l2", "divH_linf", "divE_linf"]
)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, libm only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _get():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_dft.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int]
        lib.orc_fft.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int]
        lib.orc_fft3.argtypes = [ctypes.c_int] * 3 + [dp, ctypes.c_int]
        lib.orc_wavenumbers.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        lib.orc_dmatrix.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        lib.orc_deriv.argtypes = [ctypes.c_int] * 3 + [dp, ctypes.c_int, dp, dp]
        lib.orc_coefficients.argtypes = [ctypes.c_double] * 4 + [dp, dp]
        lib.orc_coefficients.restype = None
        lib.orc_propagator.argtypes = [ctypes.c_double] * 6 + [dp]
        lib.orc_propagator.restype = None
        lib.orc_step.argtypes = ([ctypes.c_int] * 3 + [dp] + [ctypes.c_double] * 3
                                 + [ctypes.c_long, dp, dp, dp])
        lib.orc_invariants.argtypes = [ctypes.c_int] * 3 + [dp, ctypes.c_double, ctypes.c_double,
                                                           dp, dp, dp]
        lib.orc_symplectic.argtypes = [ctypes.c_int] * 3 + [dp] * 4
        lib.orc_symplectic.restype = ctypes.c_double
        lib.orc_drift_scales.argtypes = [ctypes.c_int] * 3 + [dp, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        for name in ("orc_dft", "orc_fft", "orc_fft3", "orc_wavenumbers", "orc_dmatrix",
                     "orc_deriv", "orc_step", "orc_invariants", "orc_drift_scales"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed (code {rc})")


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128))


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _dom(domain) -> np.ndarray:
    d = _f64(domain).reshape(-1)
    if d.size != 6:
        raise ValueError("domain must be (xL, xR, yL, yR, zL, zR)")
    return d


def dft(x, sign: int = -1) -> np.ndarray:
    """O(n^2) DFT, out[k] = sum_j x[j] exp(sign 2 pi i jk/n) (unnormalised)."""
    x = _c128(x)
    out = np.empty_like(x)
    _check(_get().orc_dft(x.size, _p(x.view(np.float64)), _p(out.view(np.float64)), sign), "dft")
    return out


def fft(x, sign: int = -1) -> np.ndarray:
    """The oracle's own mixed-radix FFT (unnormalised)."""
    x = _c128(x)
    out = np.empty_like(x)
    _check(_get().orc_fft(x.size, _p(x.view(np.float64)), _p(out.view(np.float64)), sign), "fft")
    return out


def fft3(a, sign: int = -1) -> np.ndarray:
    """F_{Nz} (x) F_{Ny} (x) F_{Nx} on an [nz, ny, nx] array; sign=+1 is the inverse with 1/N_S."""
    a = _c128(a).copy()
    nz, ny, nx = a.shape
    _check(_get().orc_fft3(nx, ny, nz, _p(a.view(np.float64)), sign), "fft3")
    return a


def wavenumbers(n: int, length: float) -> np.ndarray:
    out = np.empty(n)
    _check(_get().orc_wavenumbers(n, float(length), _p(out)), "wavenumbers")
    return out


def dmatrix(n: int, length: float) -> np.ndarray:
    out = np.empty((n, n))
    _check(_get().orc_dmatrix(n, float(length), _p(out)), "dmatrix")
    return out


def deriv(f, domain, axis: int) -> np.ndarray:
    """D_1, D_2 or D_3 (axis 0, 1, 2) applied to an [nz, ny, nx] real array."""
    f = _f64(f)
    nz, ny, nx = f.shape
    out = np.empty_like(f)
    d = _dom(domain)
    _check(_get().orc_deriv(nx, ny, nz, _p(d), axis, _p(f), _p(out)), "deriv")
    return out


def coefficients(b, kappa: float):
    """(c11, c12, c13, c22, c23, c33), (s12, s13, s23)/i of Prop. 2.2 for one wavevector."""
    c = np.empty(6)
    s = np.empty(3)
    _get().orc_coefficients(float(b[0]), float(b[1]), float(b[2]), float(kappa), _p(c), _p(s))
    return c, s


def propagator(b, t: float, mu: float, eps: float) -> np.ndarray:
    """6x6 complex map (H^, E^)(0) -> (H^, E^)(t) for one wavevector (Alg. 2 step 4)."""
    out = np.empty((6, 6), dtype=np.complex128)
    _get().orc_propagator(float(b[0]), float(b[1]), float(b[2]), float(t), float(mu), float(eps),
                          _p(out.view(np.float64)))
    return out


def step(H, E, domain, mu: float, eps: float, tau: float, nsteps: int = 1):
    """Return (H, E, max_imag) after nsteps steps of Alg. 2 with dt = tau."""
    H = _f64(H).copy()
    E = _f64(E).copy()
    if H.shape != E.shape or H.ndim != 4 or H.shape[0] != 3:
        raise ValueError("H and E must both be [3, nz, ny, nx]")
    _, nz, ny, nx = H.shape
    d = _dom(domain)
    mi = np.zeros(1)
    _check(_get().orc_step(nx, ny, nz, _p(d), float(mu), float(eps), float(tau), int(nsteps),
                           _p(H), _p(E), _p(mi)), "step")
    return H, E, float(mi[0])


def invariants(H, E, domain, mu: float, eps: float) -> dict:
    """Discrete invariants of Sec. 4, evaluated in physical space."""
    H = _f64(H)
    E = _f64(E)
    _, nz, ny, nx = H.shape
    d = _dom(domain)
    out = np.empty(NINV)
    _check(_get().orc_invariants(nx, ny, nz, _p(d), float(mu), float(eps), _p(H), _p(E), _p(out)),
           "invariants")
    return dict(zip(INV_NAMES, out.tolist()))


DRIFT_SCALE_NAMES = ("scale_H1", "scale_M1_x", "scale_M1_y", "scale_M1_z", "scale_divH", "scale_divE")


def drift_scales(H, E, domain, mu: float, eps: float) -> dict:
    """Cauchy-Schwarz bounds of H1, M1_k and the divergence norms (Thms 4.3, 4.4, 4.6)."""
    H = _f64(H)
    E = _f64(E)
    _, nz, ny, nx = H.shape
    d = _dom(domain)
    out = np.empty(len(DRIFT_SCALE_NAMES))
    _check(_get().orc_drift_scales(nx, ny, nz, _p(d), float(mu), float(eps), _p(H), _p(E), _p(out)),
           "drift_scales")
    return dict(zip(DRIFT_SCALE_NAMES, out.tolist()))


def symplectic(HU, EU, HV, EV) -> float:
    HU, EU, HV, EV = (_f64(a) for a in (HU, EU, HV, EV))
    _, nz, ny, nx = HU.shape
    return float(_get().orc_symplectic(nx, ny, nz, _p(HU), _p(EU), _p(HV), _p(EV)))
