"""Seeded synthetic initial fields for Maxwell's equations on a periodic cuboid.

This module only *builds inputs*: closed-form exact solutions sampled on the
collocation grid and seeded random divergence-free fields.  It contains none of the
scheme's arithmetic (no propagator, no invariant), and it is the one module that
feeds both the GPU library and the FP64 CPU oracle the same arrays.

Every field array is float64 ``[3, nz, ny, nx]`` with x fastest (the vector ordering
of Sec. 2.2), sampled at the collocation points x_j = x_L + (j-1) h_x (Sec. 2.2).
A domain is ``(xL, xR, yL, yR, zL, zR)``.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi
CUBE_2PI = (0.0, TWO_PI, 0.0, TWO_PI, 0.0, TWO_PI)
# the base of every seed: seed = SEED_BASE + 1000 * workload + stream
SEED_BASE = 2210_06232


def grid(shape, domain):
    """Collocation points (X, Y, Z), each [nz, ny, nx] (Sec. 2.2, Def. 2.3 step 1)."""
    nx, ny, nz = shape
    xl, xr, yl, yr, zl, zr = domain
    x = xl + np.arange(nx) * ((xr - xl) / nx)
    y = yl + np.arange(ny) * ((yr - yl) / ny)
    z = zl + np.arange(nz) * ((zr - zl) / nz)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


# ----------------------------------------------------------------------------------
# closed-form exact solutions
# ----------------------------------------------------------------------------------

def example1(n: int, t: float, k=(1, 2, -3), mu: float = 1.0, eps: float = 1.0):
    """Standing wave of the paper's first numerical example (Sec. 5.1), on [0, 2]^3.

    omega = |k| / sqrt(eps mu); the E amplitudes are (k_y - k_z)/(eps omega) etc.
    (the printed eps sqrt(mu) omega agrees with this at mu = 1, the value used there).
    The field solves (1.1) when k_x + k_y + k_z = 0, as for k = (1, 2, -3).
    """
    kx, ky, kz = k
    dom = (0.0, 2.0, 0.0, 2.0, 0.0, 2.0)
    X, Y, Z = grid((n, n, n), dom)
    om = math.sqrt((kx * kx + ky * ky + kz * kz) / (eps * mu))
    pi = math.pi
    ct, st = math.cos(om * pi * t), math.sin(om * pi * t)
    cx, sx = np.cos(kx * pi * X), np.sin(kx * pi * X)
    cy, sy = np.cos(ky * pi * Y), np.sin(ky * pi * Y)
    cz, sz = np.cos(kz * pi * Z), np.sin(kz * pi * Z)
    a = eps * om
    E = np.stack([(ky - kz) / a * ct * cx * sy * sz,
                  (kz - kx) / a * ct * sx * cy * sz,
                  (kx - ky) / a * ct * sx * sy * cz])
    H = np.stack([st * sx * cy * cz, st * cx * sy * cz, st * cx * cy * sz])
    return H, E, dom


def example2(n: int, t: float):
    """Travelling wave of the paper's second numerical example (Sec. 5.2), [0, 1]^3, mu = eps = 1."""
    dom = (0.0, 1.0, 0.0, 1.0, 0.0, 1.0)
    X, Y, Z = grid((n, n, n), dom)
    ex = np.cos(2 * math.pi * (X + Y + Z) - 2 * math.sqrt(3.0) * math.pi * t)
    E = np.stack([ex, -2.0 * ex, ex])
    H = np.stack([math.sqrt(3.0) * ex, np.zeros_like(ex), -math.sqrt(3.0) * ex])
    return H, E, dom


def standing_wave(n: int, t: float, mu: float = 1.0, eps: float = 1.0, t0: float = 0.0):
    """Divergence-free standing wave on [0, 2 pi]^3 built from
    A = (cos x sin y sin z, sin x cos y sin z, -2 sin x sin y cos z), which satisfies
    div A = 0 and curl curl A = 3 A.  With omega = sqrt(3/(mu eps)) and the norm
    s = sqrt(3/4) (so that <A/s, A/s>_N = 1):
        H(t) = cos(omega (t + t0)) A / s,
        E(t) = sin(omega (t + t0)) curl A / (eps omega s),
    curl A = 3 (-sin x cos y cos z, cos x sin y cos z, 0).
    """
    X, Y, Z = grid((n, n, n), CUBE_2PI)
    s = math.sqrt(0.75)
    om = math.sqrt(3.0 / (mu * eps))
    ph = om * (t + t0)
    A = np.stack([np.cos(X) * np.sin(Y) * np.sin(Z),
                  np.sin(X) * np.cos(Y) * np.sin(Z),
                  -2.0 * np.sin(X) * np.sin(Y) * np.cos(Z)])
    cA = 3.0 * np.stack([-np.sin(X) * np.cos(Y) * np.cos(Z),
                         np.cos(X) * np.sin(Y) * np.cos(Z),
                         np.zeros_like(X)])
    H = math.cos(ph) * A / s
    E = math.sin(ph) * cA / (eps * om * s)
    return H, E, CUBE_2PI


def plane_wave(shape, domain, m, e, t: float, mu: float = 1.0, eps: float = 1.0,
               phase: float = 0.0):
    """E = e cos(k.x - omega t + phase), H = (k x e)/(mu omega) cos(...), where
    k = (2 pi m_w / L_w) for integer mode numbers m and e . k = 0, omega = |k|/sqrt(mu eps).
    This solves (1.1) exactly for any mu, eps > 0."""
    L = np.array([domain[1] - domain[0], domain[3] - domain[2], domain[5] - domain[4]])
    kvec = TWO_PI * np.asarray(m, dtype=np.float64) / L
    e = np.asarray(e, dtype=np.float64)
    if abs(float(kvec @ e)) > 1e-12 * max(1.0, float(np.linalg.norm(kvec) * np.linalg.norm(e))):
        raise ValueError("polarisation e must be orthogonal to k")
    om = float(np.linalg.norm(kvec)) / math.sqrt(mu * eps)
    X, Y, Z = grid(shape, domain)
    xl, yl, zl = domain[0], domain[2], domain[4]
    arg = kvec[0] * (X - xl) + kvec[1] * (Y - yl) + kvec[2] * (Z - zl) - om * t + phase
    c = np.cos(arg)
    h = np.cross(kvec, e) / (mu * om)
    E = np.stack([e[i] * c for i in range(3)])
    H = np.stack([h[i] * c for i in range(3)])
    return H, E


# ----------------------------------------------------------------------------------
# seeded random divergence-free fields
# ----------------------------------------------------------------------------------

def _signed_modes(n: int) -> np.ndarray:
    """Integer mode numbers 0, 1, ..., n/2 - 1, -n/2, ..., -1 (numpy FFT order)."""
    return np.fft.fftfreq(n, d=1.0 / n)


def random_divfree(shape, domain, seed: int, p: float = 2.0, kcut: float | None = None,
                   norm: float = 1.0) -> np.ndarray:
    """A seeded real, band-limited, divergence-free field [3, nz, ny, nx].

    Recipe: real white noise per component -> FFT -> multiply by
    A(|k|) = (1 + |k|^2)^(-p) on 0 < |k| <= kcut (physical wavenumbers k_w = 2 pi m_w/L_w,
    default kcut = min_w(2 pi N_w / L_w)/3) -> project onto the plane orthogonal to k
    -> inverse FFT -> real part -> scale so that the grid mean of |F|^2 equals norm.
    Because |k| <= N/3 per axis, no retained mode touches a Nyquist index, so the
    field is divergence-free for the spectral derivative too.
    """
    nx, ny, nz = shape
    L = (domain[1] - domain[0], domain[3] - domain[2], domain[5] - domain[4])
    if kcut is None:
        kcut = min(TWO_PI * nx / L[0], TWO_PI * ny / L[1], TWO_PI * nz / L[2]) / 3.0
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((3, nz, ny, nx))
    F = np.fft.fftn(noise, axes=(1, 2, 3))
    kx = TWO_PI * _signed_modes(nx) / L[0]
    ky = TWO_PI * _signed_modes(ny) / L[1]
    kz = TWO_PI * _signed_modes(nz) / L[2]
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    k2 = KX * KX + KY * KY + KZ * KZ
    kk = np.sqrt(k2)
    amp = np.where((kk > 0) & (kk <= kcut), (1.0 + k2) ** (-p), 0.0)
    F *= amp
    # transverse projection F - k (k . F)/|k|^2
    safe = np.where(k2 > 0, k2, 1.0)
    kdotF = (KX * F[0] + KY * F[1] + KZ * F[2]) / safe
    F[0] -= KX * kdotF
    F[1] -= KY * kdotF
    F[2] -= KZ * kdotF
    f = np.fft.ifftn(F, axes=(1, 2, 3)).real
    ms = float(np.mean(np.sum(f * f, axis=0)))
    if ms <= 0:
        raise ValueError("empty spectrum: kcut too small for this grid")
    return np.ascontiguousarray(f * math.sqrt(norm / ms))


def random_fields(shape, domain, workload: int, p: float = 2.0, kcut: float | None = None):
    """(H, E) drawn independently, seeds SEED_BASE + 1000 * workload + {0, 1}."""
    H = random_divfree(shape, domain, SEED_BASE + 1000 * workload + 0, p=p, kcut=kcut)
    E = random_divfree(shape, domain, SEED_BASE + 1000 * workload + 1, p=p, kcut=kcut)
    return H, E


def white_noise_fields(shape, seed: int):
    """Unstructured real fields (not divergence-free, full spectrum including Nyquist
    indices) for transform parity and edge cases."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    H = rng.standard_normal((3, nz, ny, nx))
    E = rng.standard_normal((3, nz, ny, nx))
    return H, E


def upsample_bandlimited(F, fine_shape, workers: int | None = None) -> np.ndarray:
    """The trigonometric interpolant of a real grid field [3, nz, ny, nx] sampled on a
    finer grid (fine_shape = (Nx, Ny, Nz), each a multiple of the coarse size), by
    zero-padding its spectrum.  The coarse field must carry nothing at its Nyquist
    indices (the random fields above never do); its values at the shared points are
    then reproduced up to rounding, and the fine field is band-limited to the coarse
    grid's modes.  Used to build embedding inputs: a band-limited field evolves the same
    on both grids, so the fine solution at the shared points is the coarse one."""
    import os

    import scipy.fft as sfft

    F = np.asarray(F, dtype=np.float64)
    _, nz, ny, nx = F.shape
    Nx, Ny, Nz = fine_shape
    if Nx % nx or Ny % ny or Nz % nz:
        raise ValueError("fine grid sizes must be multiples of the coarse ones")
    w = workers or max(1, min(16, os.cpu_count() or 1))
    # signed coarse indices (Nyquist dropped) -> positions on the fine grid
    zi = np.r_[0:nz // 2, nz // 2 + 1:nz]
    yi = np.r_[0:ny // 2, ny // 2 + 1:ny]
    zf = np.where(zi < nz // 2, zi, Nz - (nz - zi))
    yf = np.where(yi < ny // 2, yi, Ny - (ny - yi))
    out = np.empty((3, Nz, Ny, Nx))
    scale = (Nx * Ny * Nz) / (nx * ny * nz)
    for c in range(3):
        G = sfft.rfftn(F[c], workers=w)
        Gp = np.zeros((Nz, Ny, Nx // 2 + 1), dtype=np.complex128)
        Gp[np.ix_(zf, yf, np.arange(nx // 2))] = G[np.ix_(zi, yi, np.arange(nx // 2))]
        out[c] = sfft.irfftn(Gp, s=(Nz, Ny, Nx), workers=w) * scale
        del G, Gp
    return out
