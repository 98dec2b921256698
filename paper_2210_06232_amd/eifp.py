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
EIFP_ERR_CANCELLED = 7

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


EIFP_SERVER_DRY_RUN = 1
EIFP_SERVER_NO_GRAPHS = 2
EIFP_SERVER_SERIAL = 4
EIFP_REQ_KEEP_RESULT = 1
EIFP_REQ_NO_SNAPSHOT = 2
EIFP_REQ_ANCHORED = 4
EIFP_EV_OUTPUT = 0
EIFP_EV_DONE = 1
EIFP_EV_ERROR = 2
EVENT_KINDS = {EIFP_EV_OUTPUT: "output", EIFP_EV_DONE: "done", EIFP_EV_ERROR: "error"}


class eifp_request(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("dom", eifp_domain),
        ("mu", ctypes.c_double), ("eps", ctypes.c_double), ("tau", ctypes.c_double),
        ("nsteps", ctypes.c_longlong), ("cadence", ctypes.c_longlong),
        ("prec", ctypes.c_int),
        ("H0", ctypes.POINTER(ctypes.c_double)), ("E0", ctypes.POINTER(ctypes.c_double)),
        ("user_tag", ctypes.c_ulonglong),
        ("flags", ctypes.c_int),
    ]


class eifp_event(ctypes.Structure):
    _fields_ = [
        ("user_tag", ctypes.c_ulonglong),
        ("req_id", ctypes.c_longlong),
        ("kind", ctypes.c_int),
        ("status", ctypes.c_int),
        ("step", ctypes.c_longlong),
        ("inv", eifp_invariant_set),
        ("t_arrive", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_event", ctypes.c_double),
    ]


class eifp_server_stat_set(ctypes.Structure):
    _fields_ = [(n, ctypes.c_longlong) for n in
                ("submitted", "admitted", "completed", "failed", "queued", "running", "peak_running")] + \
               [(n, ctypes.c_double) for n in ("p50_s", "p99_s", "mean_s", "max_s", "point_steps", "wall_s",
                                                "point_steps_per_s")] + \
               [(n, ctypes.c_longlong) for n in ("bytes_in_use", "peak_bytes", "budget_bytes", "chunks")] + \
               [("mean_batch", ctypes.c_double), ("cancelled", ctypes.c_longlong)]


class eifp_invariant_ext_set(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double),
        ("steps_done", ctypes.c_longlong),
        ("e2", ctypes.c_double),
        ("e3", ctypes.c_double * 3),
        ("e4", ctypes.c_double * 3),
        ("h2", ctypes.c_double),
        ("scale_helicity", ctypes.c_double),
        ("scale_momentum", ctypes.c_double * 3),
        ("scale_div_h", ctypes.c_double),
        ("scale_div_e", ctypes.c_double),
    ]


# every symbol the header declares, with (restype, argtypes)
_VP = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "eifp_init": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(eifp_domain), ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int, _DP, _DP, _VP]),
    "eifp_step": (ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_longlong]),
    "eifp_anchor": (ctypes.c_int, [_VP]),
    "eifp_jump": (ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_longlong]),
    "eifp_step_timed": (ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_longlong, _DP]),
    "eifp_invariants": (ctypes.c_int, [_VP, ctypes.POINTER(eifp_invariant_set)]),
    "eifp_invariants_ext": (ctypes.c_int, [_VP, ctypes.POINTER(eifp_invariant_ext_set)]),
    "eifp_fields": (ctypes.c_int, [_VP, _DP, _DP]),
    "eifp_fields_device": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int]),
    "eifp_spectrum": (ctypes.c_int, [_VP, _DP]),
    "eifp_sync": (ctypes.c_int, [_VP]),
    "eifp_stream": (_VP, [_VP]),
    "eifp_device_bytes": (ctypes.c_longlong, [_VP]),
    "eifp_destroy": (ctypes.c_int, [_VP]),
    "eifp_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "eifp_last_error": (ctypes.c_char_p, []),
    "eifp_server_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_longlong, ctypes.c_int, ctypes.c_int]),
    "eifp_server_footprint": (ctypes.c_longlong, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_int]),
    "eifp_server_submit": (ctypes.c_int, [_VP, ctypes.POINTER(eifp_request), ctypes.POINTER(ctypes.c_longlong)]),
    "eifp_server_poll": (ctypes.c_int, [_VP, ctypes.POINTER(eifp_event), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "eifp_server_fields": (ctypes.c_int, [_VP, ctypes.c_longlong, _DP, _DP, ctypes.POINTER(ctypes.c_longlong)]),
    "eifp_server_release": (ctypes.c_int, [_VP, ctypes.c_longlong]),
    "eifp_server_cancel": (ctypes.c_int, [_VP, ctypes.c_longlong]),
    "eifp_server_stats": (ctypes.c_int, [_VP, ctypes.POINTER(eifp_server_stat_set)]),
    "eifp_server_drain": (ctypes.c_int, [_VP, ctypes.c_int]),
    "eifp_server_destroy": (ctypes.c_int, [_VP]),
    "eifp_step_noalloc": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(eifp_domain),
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_longlong, _VP, _VP]),
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


def eifp_anchor(handle):
    _check(load().eifp_anchor(handle), "eifp_anchor")


def eifp_jump(handle, tau, nsteps=1):
    _check(load().eifp_jump(handle, float(tau), int(nsteps)), "eifp_jump")


def eifp_step_timed(handle, tau, nsteps=1) -> dict:
    out = np.zeros(6)
    _check(load().eifp_step_timed(handle, float(tau), int(nsteps), _dp(out)), "eifp_step_timed")
    return dict(zip(PASS_NAMES, out.tolist()))


def _inv_dict(inv: eifp_invariant_set) -> dict:
    return {"t": inv.t, "steps_done": inv.steps_done, "energy": inv.energy, "helicity": inv.helicity,
            "momentum": list(inv.momentum), "div_h_l2": inv.div_h_l2, "div_e_l2": inv.div_e_l2}


def eifp_invariants(handle) -> dict:
    inv = eifp_invariant_set()
    _check(load().eifp_invariants(handle, ctypes.byref(inv)), "eifp_invariants")
    return _inv_dict(inv)


def eifp_invariants_ext(handle) -> dict:
    x = eifp_invariant_ext_set()
    _check(load().eifp_invariants_ext(handle, ctypes.byref(x)), "eifp_invariants_ext")
    return {"t": x.t, "steps_done": x.steps_done, "E2": x.e2, "E3": list(x.e3), "E4": list(x.e4), "H2": x.h2,
            "scale_helicity": x.scale_helicity, "scale_momentum": list(x.scale_momentum),
            "scale_div_h": x.scale_div_h, "scale_div_e": x.scale_div_e}


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


def eifp_step_noalloc(fields_ptr: int, shape, domain, mu, eps, prec, tau, nsteps=1, inv_ptr: int = 0,
                      stream: int = 0):
    """Step a caller-owned device state [6, nz, ny, nx] (in the working precision) in
    place, with no device allocation; shape = (nx, ny, nz).  Enqueues only."""
    nx, ny, nz = shape
    p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    dom = eifp_domain(*[float(v) for v in domain])
    _check(load().eifp_step_noalloc(fields_ptr or None, int(nx), int(ny), int(nz), ctypes.byref(dom), float(mu),
                                    float(eps), p, float(tau), int(nsteps), inv_ptr or None, stream or None),
           "eifp_step_noalloc")


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

    def anchor(self):
        eifp_anchor(self.handle)
        return self

    def jump(self, tau, nsteps=1):
        eifp_jump(self.handle, tau, nsteps)
        return self

    def step_timed(self, tau, nsteps=1) -> dict:
        return eifp_step_timed(self.handle, tau, nsteps)

    def invariants(self) -> dict:
        return eifp_invariants(self.handle)

    def invariants_ext(self) -> dict:
        return eifp_invariants_ext(self.handle)

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


# ----------------------------------------------------------------------------------
# serving
# ----------------------------------------------------------------------------------

def eifp_server_create(budget_bytes, max_batch=32, flags=0) -> int:
    h = _VP()
    _check(load().eifp_server_create(ctypes.byref(h), int(budget_bytes), int(max_batch), int(flags)),
           "eifp_server_create")
    return h.value


def eifp_server_footprint(nx, ny, nz, prec, flags=0) -> int:
    p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    return int(load().eifp_server_footprint(nx, ny, nz, p, int(flags)))


def eifp_server_submit(handle, H0, E0, domain, mu, eps, tau, nsteps, cadence=0, prec="fp64", tag=0,
                       flags=0) -> int:
    H0 = _field(H0)
    _, nz, ny, nx = H0.shape
    E0 = _field(E0, H0.shape)
    p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    rq = eifp_request(nx, ny, nz, eifp_domain(*[float(v) for v in domain]), float(mu), float(eps), float(tau),
                      int(nsteps), int(cadence), p, _dp(H0), _dp(E0), int(tag), int(flags))
    rid = ctypes.c_longlong()
    _check(load().eifp_server_submit(handle, ctypes.byref(rq), ctypes.byref(rid)), "eifp_server_submit")
    return rid.value


def eifp_server_poll(handle, max_events=256, wait_ms=0) -> list:
    buf = (eifp_event * max(1, max_events))()
    n = ctypes.c_int()
    _check(load().eifp_server_poll(handle, buf, int(max_events), ctypes.byref(n), int(wait_ms)),
           "eifp_server_poll")
    out = []
    for e in buf[:n.value]:
        out.append({"tag": e.user_tag, "req_id": e.req_id, "kind": EVENT_KINDS.get(e.kind, e.kind),
                    "status": e.status, "step": e.step, "inv": _inv_dict(e.inv), "t_arrive": e.t_arrive,
                    "t_admit": e.t_admit, "t_event": e.t_event})
    return out


def eifp_server_fields(handle, req_id, shape):
    """Returns (H, E, step): the fields of a request and the step count they are at."""
    nx, ny, nz = shape
    H = np.empty((3, nz, ny, nx))
    E = np.empty((3, nz, ny, nx))
    step = ctypes.c_longlong()
    _check(load().eifp_server_fields(handle, int(req_id), _dp(H), _dp(E), ctypes.byref(step)),
           "eifp_server_fields")
    return H, E, step.value


def eifp_server_release(handle, req_id):
    _check(load().eifp_server_release(handle, int(req_id)), "eifp_server_release")


def eifp_server_cancel(handle, req_id):
    _check(load().eifp_server_cancel(handle, int(req_id)), "eifp_server_cancel")


def eifp_server_stats(handle) -> dict:
    s = eifp_server_stat_set()
    _check(load().eifp_server_stats(handle, ctypes.byref(s)), "eifp_server_stats")
    return {name: getattr(s, name) for name, _ in s._fields_}


def eifp_server_drain(handle, timeout_ms=-1):
    _check(load().eifp_server_drain(handle, int(timeout_ms)), "eifp_server_drain")


def eifp_server_destroy(handle):
    _check(load().eifp_server_destroy(handle), "eifp_server_destroy")


class Server:
    """Owns one library server.  ``Server(budget_bytes, max_batch=32, flags=0)``."""

    def __init__(self, budget_bytes, max_batch=32, flags=0):
        self.handle = eifp_server_create(budget_bytes, max_batch, flags)

    def submit(self, H0, E0, domain, mu=1.0, eps=1.0, tau=0.1, nsteps=1, cadence=0, prec="fp64", tag=0,
               flags=0) -> int:
        return eifp_server_submit(self.handle, H0, E0, domain, mu, eps, tau, nsteps, cadence, prec, tag, flags)

    def poll(self, max_events=256, wait_ms=0) -> list:
        return eifp_server_poll(self.handle, max_events, wait_ms)

    def fields(self, req_id, shape):
        return eifp_server_fields(self.handle, req_id, shape)

    def release(self, req_id):
        eifp_server_release(self.handle, req_id)

    def cancel(self, req_id):
        """End a queued or running request (its last event: error, status CANCELLED)."""
        eifp_server_cancel(self.handle, req_id)

    def stats(self) -> dict:
        return eifp_server_stats(self.handle)

    def drain(self, timeout_ms=-1):
        eifp_server_drain(self.handle, timeout_ms)

    def close(self):
        if self.handle:
            eifp_server_destroy(self.handle)
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
