"""Pins of the oracle's full step (Def. 2.3, Alg. 1-2) against exact solutions and the
paper's printed accuracy, plus composition properties of the exact propagator."""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2210_06232_amd import inputs
from tests.helpers import errors, read_golden, energy_rel_error


@pytest.mark.parametrize("example", [1, 2])
def test_paper_examples_one_jump_beat_printed_errors(example):
    # One step with dt = t_end reproduces the exact solution at least as well as the
    # paper's own runs (Tables "error s2" and "error s").
    rows = read_golden(f"example{example}_solution_errors.txt")
    make = inputs.example1 if example == 1 else inputs.example2
    for n, t_end, linf_paper, l2_paper in rows:
        n = int(n)
        H0, E0, dom = make(n, 0.0)
        Hx, Ex, _ = make(n, t_end)
        H, E, mi = orc.step(H0, E0, dom, 1.0, 1.0, t_end, 1)
        linf, l2 = errors(H, E, Hx, Ex)
        assert linf <= linf_paper, (n, t_end, linf, linf_paper)
        assert l2 <= l2_paper, (n, t_end, l2, l2_paper)
        assert mi < 1e-13


def test_example2_many_small_steps():
    H0, E0, dom = inputs.example2(8, 0.0)
    Hx, Ex, _ = inputs.example2(8, 5.0)
    H, E, _ = orc.step(H0, E0, dom, 1.0, 1.0, 0.05, 100)
    linf, l2 = errors(H, E, Hx, Ex)
    assert linf < 1e-13 and l2 < 1e-13


@pytest.mark.parametrize("mu,eps,t0", [(1.0, 1.0, 0.0), (1.0, 1.0, 0.3), (1.0, 2.0, 0.0), (2.0, 0.5, 0.3)])
def test_standing_wave_16cubed_100_steps(mu, eps, t0):
    # the 16^3 standing-wave workload: tau = 0.01, 100 steps, error at round-off
    H0, E0, dom = inputs.standing_wave(16, 0.0, mu, eps, t0)
    Hx, Ex, _ = inputs.standing_wave(16, 1.0, mu, eps, t0)
    H, E, _ = orc.step(H0, E0, dom, mu, eps, 0.01, 100)
    assert energy_rel_error(H, E, Hx, Ex, mu, eps) < 1e-13


@pytest.mark.parametrize("tau,n", [(0.05, 40), (3.7, 3)])
def test_plane_wave_noncubic_box_any_mu_eps(tau, n):
    shape = (12, 8, 16)
    dom = (0.0, 2 * math.pi, -1.0, 4 * math.pi - 1.0, 0.5, 2.5)
    mu, eps = 1.3, 0.7
    m = (2, -1, 3)
    L = np.array([dom[1] - dom[0], dom[3] - dom[2], dom[5] - dom[4]])
    k = 2 * math.pi * np.array(m) / L
    e = np.cross(k, [0.3, 1.0, -0.2])
    H0, E0 = inputs.plane_wave(shape, dom, m, e, 0.0, mu, eps, phase=0.4)
    Hx, Ex = inputs.plane_wave(shape, dom, m, e, tau * n, mu, eps, phase=0.4)
    H, E, _ = orc.step(H0, E0, dom, mu, eps, tau, n)
    assert energy_rel_error(H, E, Hx, Ex, mu, eps) < 1e-13


def _random_state(shape, dom, seed):
    H = inputs.random_divfree(shape, dom, seed, p=1.0)
    E = inputs.random_divfree(shape, dom, seed + 1, p=1.0)
    return H, E


def test_group_property_and_reversibility():
    shape = (12, 8, 16)
    dom = (0.0, 2 * math.pi, 0.0, 4 * math.pi, 0.0, 2 * math.pi)
    H0, E0 = inputs.white_noise_fields(shape, 11)      # includes Nyquist content
    mu, eps = 1.0, 2.0
    H1, E1, _ = orc.step(H0, E0, dom, mu, eps, 0.37, 50)
    H2, E2, _ = orc.step(H0, E0, dom, mu, eps, 0.37 * 50, 1)
    assert energy_rel_error(H1, E1, H2, E2, mu, eps) < 1e-12
    H3, E3, _ = orc.step(H1, E1, dom, mu, eps, -0.37, 50)
    assert energy_rel_error(H3, E3, H0, E0, mu, eps) < 1e-12
    H4, E4, _ = orc.step(H0, E0, dom, mu, eps, 0.0, 3)
    assert energy_rel_error(H4, E4, H0, E0, mu, eps) < 1e-15


def test_nyquist_modes_follow_the_zeroed_wavenumber():
    # a field living only on the x-Nyquist index: Omega_x = 0 there, so with no y/z
    # dependence the mode is held fixed (Psi = 0) for any step.
    n = 8
    X, Y, Z = inputs.grid((n, n, n), inputs.CUBE_2PI)
    f = np.cos(4 * X)
    H = np.stack([np.zeros_like(f), f, 2 * f])
    E = np.stack([np.zeros_like(f), -f, 0.5 * f])
    H1, E1, _ = orc.step(H, E, inputs.CUBE_2PI, 1.0, 1.0, 0.9, 1)
    np.testing.assert_allclose(H1, H, atol=1e-14)
    np.testing.assert_allclose(E1, E, atol=1e-14)


def test_embedding_coarse_in_fine_grid():
    # A trigonometric polynomial of degree <= 2 per axis evolves identically on 8^3 and
    # on 16^3 (the scheme is exact for band-limited data), so the fine result sampled
    # at the coarse points equals the coarse result.
    dom = (0.0, 2 * math.pi, 0.0, 4 * math.pi, 0.0, 2 * math.pi)
    rng = np.random.default_rng(5)
    nc, nf = 8, 16

    def field(n):
        X, Y, Z = inputs.grid((n, n, n), dom)
        out = np.zeros((3, n, n, n))
        for c in range(3):
            for (a, b, d) in [(1, 0, 2), (0, 1, -1), (2, -2, 1), (1, 1, 1)]:
                amp, ph = r[c][(a, b, d)]
                out[c] += amp * np.cos(a * X + b * Y / 2 + d * Z + ph)
        return out

    r = [{m: (rng.standard_normal(), rng.uniform(0, 6)) for m in
          [(1, 0, 2), (0, 1, -1), (2, -2, 1), (1, 1, 1)]} for _ in range(3)]
    Hc, Ec = field(nc), 0.5 * field(nc)[::-1]
    Hf, Ef = field(nf), 0.5 * field(nf)[::-1]
    Hc1, Ec1, _ = orc.step(Hc, Ec, dom, 1.0, 1.5, 0.7, 3)
    Hf1, Ef1, _ = orc.step(Hf, Ef, dom, 1.0, 1.5, 0.7, 3)
    np.testing.assert_allclose(Hf1[:, ::2, ::2, ::2], Hc1, atol=1e-13)
    np.testing.assert_allclose(Ef1[:, ::2, ::2, ::2], Ec1, atol=1e-13)


def test_rejects_bad_arguments():
    H, E = inputs.white_noise_fields((4, 4, 4), 0)
    with pytest.raises(ValueError):
        orc.step(H, E, inputs.CUBE_2PI, -1.0, 1.0, 0.1, 1)
    with pytest.raises(ValueError):
        orc.step(H, E, inputs.CUBE_2PI, 1.0, 1.0, float("nan"), 1)
    H5, E5 = inputs.white_noise_fields((5, 4, 4), 0)
    with pytest.raises(ValueError):
        orc.step(H5, E5, inputs.CUBE_2PI, 1.0, 1.0, 0.1, 1)
