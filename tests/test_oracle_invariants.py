"""Pins of the oracle's discrete invariants (Sec. 4): closed-form values on simple
fields, conservation under the scheme (Thms 4.1, 4.3-4.6), structural identities, and
the paper's printed energy/divergence errors for its two examples."""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2210_06232_amd import inputs
from tests.helpers import read_golden

CUBE = inputs.CUBE_2PI


def test_closed_form_values_circular_field():
    # H = (cos z, sin z, 0): curl H = -H, <H, H>_N = 1, so with E = 0
    # E1 = mu/2, H1 = -1/(2 eps), E3_z = mu/2, E5 = 0, divergence 0.
    n = 8
    X, Y, Z = inputs.grid((n, n, n), CUBE)
    H = np.stack([np.cos(Z), np.sin(Z), np.zeros_like(Z)])
    E = np.zeros_like(H)
    mu, eps = 1.7, 0.6
    inv = orc.invariants(H, E, CUBE, mu, eps)
    assert abs(inv["E1"] - mu / 2) < 1e-14
    assert abs(inv["H1"] + 1 / (2 * eps)) < 1e-14
    assert abs(inv["E3_z"] - mu / 2) < 1e-14
    assert abs(inv["E3_x"]) < 1e-14 and abs(inv["E3_y"]) < 1e-14
    # d/dt E = (1/eps) curl H = -H/eps, d/dt H = 0: E2 = eps/2 <H,H>/eps^2 = 1/(2 eps)
    assert abs(inv["E2"] - 1 / (2 * eps)) < 1e-14
    for k in "xyz":
        assert abs(inv[f"E5_{k}"]) < 1e-15 and abs(inv[f"E6_{k}"]) < 1e-15
    assert inv["divH_linf"] < 1e-14 and inv["divE_linf"] < 1e-14


def test_closed_form_momentum_and_divergence():
    # H = h cos x, E = e sin x: D_1 E = e cos x, so M1_x = h.e/2 and M2_x = -h.e/2.
    n = 8
    X, Y, Z = inputs.grid((n, n, n), CUBE)
    h = np.array([0.0, 1.0, 2.0])
    e = np.array([0.5, 2.0, -1.0])
    H = np.stack([hc * np.cos(X) for hc in h])
    E = np.stack([ec * np.sin(X) for ec in e])
    mu, eps = 2.0, 3.0
    inv = orc.invariants(H, E, CUBE, mu, eps)
    assert abs(inv["M1_x"] - h @ e / 2) < 1e-14
    assert abs(inv["M2_x"] + h @ e / 2) < 1e-14
    for k in "yz":
        assert abs(inv[f"M1_{k}"]) < 1e-14 and abs(inv[f"M2_{k}"]) < 1e-14
    # div(mu H) = mu h_x (-sin x) = 0 since h_x = 0; div(eps E) = eps e_x cos x
    assert inv["divH_linf"] < 1e-13
    assert abs(inv["divE_linf"] - eps * e[0]) < 1e-13
    assert abs(inv["divE_l2"] - eps * e[0] / math.sqrt(2)) < 1e-13


def test_plane_wave_energy_family():
    # For E = e cos(k.x), H = (k x e)/(mu w) cos(k.x): E1 = (mu|h|^2 + eps|e|^2)/4,
    # E2 = w^2 E1, E3_w = k_w^2 E1, E4_w = w^2 k_w^2 E1 (every derivative multiplies the
    # amplitude by the corresponding frequency; the mean of cos^2 and sin^2 is 1/2).
    shape = (8, 8, 8)
    dom = (0.0, 2 * math.pi, 0.0, 4 * math.pi, 0.0, 2 * math.pi)
    m = (1, 2, -1)
    k = np.array([1.0, 1.0, -1.0])
    e = np.array([1.0, 0.0, 1.0])
    mu, eps = 1.0, 2.0
    H, E = inputs.plane_wave(shape, dom, m, e, 0.0, mu, eps)
    w = np.linalg.norm(k) / math.sqrt(mu * eps)
    h = np.cross(k, e) / (mu * w)
    E1 = (mu * h @ h + eps * e @ e) / 4
    inv = orc.invariants(H, E, dom, mu, eps)
    assert abs(inv["E1"] - E1) < 1e-13
    assert abs(inv["E2"] - w * w * E1) < 1e-13
    for i, c in enumerate("xyz"):
        assert abs(inv[f"E3_{c}"] - k[i] ** 2 * E1) < 1e-13
        assert abs(inv[f"E4_{c}"] - w * w * k[i] ** 2 * E1) < 1e-13
    assert abs(inv["H1"]) < 1e-13          # linear polarisation carries no helicity


@pytest.mark.parametrize("kind", ["divfree", "white"])
def test_conservation_under_the_scheme(kind):
    shape = (12, 8, 16)
    dom = (0.0, 2 * math.pi, 0.0, 4 * math.pi, 0.0, 2 * math.pi)
    mu, eps = 1.0, 2.0
    if kind == "divfree":
        H = inputs.random_divfree(shape, dom, 3, p=1.0)
        E = inputs.random_divfree(shape, dom, 4, p=1.0)
    else:
        H, E = inputs.white_noise_fields(shape, 3)
    a = orc.invariants(H, E, dom, mu, eps)
    H1, E1, _ = orc.step(H, E, dom, mu, eps, 0.37, 20)
    b = orc.invariants(H1, E1, dom, mu, eps)
    # energy-like quantities: relative; signed ones: scaled by the energy of the same order
    scale = {k: max(abs(a[k]), 1e-300) for k in a}
    for k in ("E1", "E2") + tuple(f"E3_{c}" for c in "xyz") + tuple(f"E4_{c}" for c in "xyz"):
        assert abs(b[k] - a[k]) <= 1e-13 * scale[k], k
    e_ref = math.sqrt(a["E1"] * a["E2"])
    for k in ("H1",) + tuple(f"M1_{c}" for c in "xyz") + tuple(f"M2_{c}" for c in "xyz"):
        assert abs(b[k] - a[k]) <= 1e-13 * e_ref, k
    assert abs(b["H2"] - a["H2"]) <= 1e-13 * a["E2"] * math.sqrt(a["E2"] / a["E1"])
    # divergence: unchanged (zero for the div-free data, nonzero for white noise)
    for k in ("divH_l2", "divE_l2"):
        assert abs(b[k] - a[k]) <= 1e-13 * max(1.0, a[k]) * 10, k
    if kind == "divfree":
        assert a["divH_linf"] < 1e-13 and a["divE_linf"] < 1e-13


def test_structural_identities():
    # M2 = -M1 (B_k skew) and E5 = E6 = 0 (D_k skew) for any real fields.
    H, E = inputs.white_noise_fields((8, 6, 4), 9)
    dom = (0.0, 1.0, 0.0, 2.0, 0.0, 3.0)
    inv = orc.invariants(H, E, dom, 1.3, 0.7)
    for c in "xyz":
        assert abs(inv[f"M1_{c}"] + inv[f"M2_{c}"]) < 1e-12
        assert abs(inv[f"E5_{c}"]) < 1e-12 and abs(inv[f"E6_{c}"]) < 1e-11


def test_symplectic_form_conserved():
    # Thm 4.5: the flow preserves dE ^ dH, i.e. the bilinear form between two solutions.
    shape = (8, 8, 8)
    dom = CUBE
    mu, eps = 1.2, 0.9
    HU, EU = inputs.white_noise_fields(shape, 21)
    HV, EV = inputs.white_noise_fields(shape, 22)
    w0 = orc.symplectic(HU, EU, HV, EV)
    HU1, EU1, _ = orc.step(HU, EU, dom, mu, eps, 0.8, 5)
    HV1, EV1, _ = orc.step(HV, EV, dom, mu, eps, 0.8, 5)
    w1 = orc.symplectic(HU1, EU1, HV1, EV1)
    assert abs(w0) > 1e-3
    assert abs(w1 - w0) < 1e-13 * (1 + abs(w0))


@pytest.mark.parametrize("example", [1, 2])
def test_paper_energy_and_divergence_tables(example):
    # The paper's printed relative energy errors (<= 6e-16) and divergences (<= 4.4e-14)
    # for one jump to t_end; a correct FP64 oracle stays within a few units of round-off
    # of them.
    make = inputs.example1 if example == 1 else inputs.example2
    e_rows = read_golden(f"example{example}_energy_errors.txt")
    d_rows = read_golden("divergence_errors.txt")
    d_rows = d_rows[d_rows[:, 0] == example]
    bound_e = 2 * e_rows[:, 2:].max()
    bound_d = 4 * d_rows[:, 3:].max() + 1e-14
    for n, t_end in e_rows[:, :2]:
        H0, E0, dom = make(int(n), 0.0)
        a = orc.invariants(H0, E0, dom, 1.0, 1.0)
        H, E, _ = orc.step(H0, E0, dom, 1.0, 1.0, t_end, 1)
        b = orc.invariants(H, E, dom, 1.0, 1.0)
        for k in ("E1", "E2", "E3_x", "E4_x"):
            assert abs(b[k] - a[k]) / abs(a[k]) <= bound_e, (n, t_end, k)
        assert b["divH_linf"] <= bound_d and b["divE_linf"] <= bound_d


# ---- drift scales: Cauchy-Schwarz bounds of H1, M1_k and the divergence norms --------

def test_drift_scales_equality_cases():
    n = 8
    X, Y, Z = inputs.grid((n, n, n), CUBE)
    mu, eps = 1.7, 0.6
    zero = np.zeros((3, n, n, n))
    # circularly polarised H = (cos z, sin z, 0): Re H^ and Im H^ orthogonal, equal, and
    # their cross product along b, so |H1| reaches its bound 1/(2 eps)
    H = np.stack([np.cos(Z), np.sin(Z), np.zeros_like(Z)])
    sc = orc.drift_scales(H, zero, CUBE, mu, eps)
    inv = orc.invariants(H, zero, CUBE, mu, eps)
    assert abs(sc["scale_H1"] - 1 / (2 * eps)) < 1e-14
    assert abs(abs(inv["H1"]) - sc["scale_H1"]) < 1e-14
    # a gradient field (H^ parallel to b in every mode) reaches the divergence bound
    ph = X + 2 * Y
    H = np.stack([-np.sin(ph), -2 * np.sin(ph), 3 * np.cos(3 * Z)])
    sc = orc.drift_scales(H, H, CUBE, mu, eps)
    inv = orc.invariants(H, H, CUBE, mu, eps)
    assert abs(inv["divH_l2"] - sc["scale_divH"]) < 1e-12 * sc["scale_divH"]
    assert abs(inv["divE_l2"] - sc["scale_divE"]) < 1e-12 * sc["scale_divE"]
    # H = h cos x, E = e sin x with e parallel to h: |M1_x| = |h||e|/2 is its bound
    h = np.array([0.0, 1.0, 2.0])
    H = h[:, None, None, None] * np.cos(X)[None]
    E = 1.5 * H / np.cos(X)[None] * np.sin(X)[None]
    sc = orc.drift_scales(H, E, CUBE, mu, eps)
    inv = orc.invariants(H, E, CUBE, mu, eps)
    assert abs(sc["scale_M1_x"] - 1.5 * (h @ h) / 2) < 1e-13
    assert abs(abs(inv["M1_x"]) - sc["scale_M1_x"]) < 1e-13
    assert sc["scale_M1_y"] < 1e-14 and sc["scale_M1_z"] < 1e-14  # no E content along y or z


@pytest.mark.parametrize("seed", [1, 2])
def test_drift_scales_bound_the_invariants(seed):
    box = (0.0, 2 * math.pi, -1.0, 3.0, 0.5, 2.5)
    H, E = inputs.white_noise_fields((8, 6, 10), seed)
    mu, eps = 1.3, 0.7
    sc = orc.drift_scales(H, E, box, mu, eps)
    inv = orc.invariants(H, E, box, mu, eps)
    assert abs(inv["H1"]) <= sc["scale_H1"]
    for k in "xyz":
        assert abs(inv[f"M1_{k}"]) <= sc[f"scale_M1_{k}"]
    assert inv["divH_l2"] <= sc["scale_divH"] and inv["divE_l2"] <= sc["scale_divE"]
    # a bound, not a loose one: each is within a modest factor on white noise
    assert sc["scale_divH"] < 10 * inv["divH_l2"]


def test_helicity_scale_conserved_by_the_scheme():
    # per mode, |H^|^2/(2 eps) + |E^|^2/(2 mu) is the mode's energy over mu eps, which the
    # exact flow keeps; so the helicity scale is conserved like E1
    box = (0.0, 2 * math.pi, -1.0, 3.0, 0.5, 2.5)
    H, E = inputs.white_noise_fields((8, 6, 10), 3)
    mu, eps = 1.3, 0.7
    s0 = orc.drift_scales(H, E, box, mu, eps)["scale_H1"]
    H1, E1, _ = orc.step(H, E, box, mu, eps, 0.37, 5)
    s1 = orc.drift_scales(H1, E1, box, mu, eps)["scale_H1"]
    assert abs(s1 - s0) < 1e-13 * s0
