"""The seeded input generators: real, divergence-free (checked with the oracle's spectral
derivative), normalised, reproducible, and exact solutions of (1.1)."""
import math

import numpy as np

from oracle import oracle as orc
from paper_2210_06232_amd import inputs


def test_random_divfree_properties():
    shape = (16, 8, 12)
    dom = (0.0, 2 * math.pi, 0.0, 4 * math.pi, 0.0, 2 * math.pi)
    a = inputs.random_divfree(shape, dom, 123, p=2.0)
    b = inputs.random_divfree(shape, dom, 123, p=2.0)
    c = inputs.random_divfree(shape, dom, 124, p=2.0)
    assert a.shape == (3, 12, 8, 16) and a.dtype == np.float64
    np.testing.assert_array_equal(a, b)
    assert np.max(np.abs(a - c)) > 0.1
    assert abs(np.mean(np.sum(a * a, axis=0)) - 1.0) < 1e-12
    inv = orc.invariants(a, np.zeros_like(a), dom, 1.0, 1.0)
    assert inv["divH_linf"] < 1e-13
    # band limit: no content at or beyond N/3 along x
    F = np.fft.fftn(a[0])
    m = np.abs(np.fft.fftfreq(16, 1 / 16))
    assert np.max(np.abs(F[:, :, m > 16 / 3])) < 1e-10


def test_random_fields_seeds_follow_the_workload():
    shape = (8, 8, 8)
    H, E = inputs.random_fields(shape, inputs.CUBE_2PI, workload=1)
    H2 = inputs.random_divfree(shape, inputs.CUBE_2PI, inputs.SEED_BASE + 1000 * 1 + 0)
    np.testing.assert_array_equal(H, H2)
    assert np.max(np.abs(H - E)) > 0.1


def test_standing_wave_normalisation_and_divergence():
    H, E, dom = inputs.standing_wave(16, 0.0)
    assert abs(np.mean(np.sum(H * H, axis=0)) - 1.0) < 1e-13
    assert np.max(np.abs(E)) == 0.0
    H, E, dom = inputs.standing_wave(16, 0.0, 1.0, 2.0, t0=0.3)
    inv = orc.invariants(H, E, dom, 1.0, 2.0)
    assert inv["divH_linf"] < 1e-13 and inv["divE_linf"] < 1e-13


def test_subsampling_evaluates_the_same_field():
    # a field given on the fine grid, read at the coarse grid's points, is the same
    # trigonometric polynomial evaluated there
    from paper_2210_06232_amd import convergence
    n, m = 24, 8
    x = np.arange(n) * 2 * np.pi / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    F = np.stack([np.cos(2 * X + Y), np.sin(X - 3 * Z), np.cos(Y) * np.sin(Z)])
    xc = np.arange(m) * 2 * np.pi / m
    Zc, Yc, Xc = np.meshgrid(xc, xc, xc, indexing="ij")
    Fc = np.stack([np.cos(2 * Xc + Yc), np.sin(Xc - 3 * Zc), np.cos(Yc) * np.sin(Zc)])
    assert np.allclose(convergence.subsample(F, m), Fc, atol=1e-14)
