"""The plane pass: grids whose (y, z) plane of the six components fits in LDS step with
one workgroup per packed x column (z and y transforms, propagator, invariant partials
and the inverse transforms in one launch), the x kernel after it finalizing the
invariants.

Gates, as for the strided passes: one step against one oracle step (Def. 2.3 / Alg. 2)
at 1e-12 (FP64) and 2e-6 (FP32, from FP32-rounded input), in the energy norm and element
by element; the step's invariants against the oracle's (Sec. 4); n steps in one call
against n calls of one step, bitwise; and the invariants a plane step reports against
those the strided forward passes compute for the same state.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2210_06232_amd import inputs
from tests.helpers import elementwise_rel_error, energy_rel_error

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-6}
DOMAIN = (0.0, 2 * math.pi, -1.0, 4 * math.pi - 1.0, 0.5, 2.5)
# every pencil length of the plane pass (4 ... 32, with the factor-3 lengths) along y and
# along z, small and wide in x, up to the largest planes it takes (576 points: 24 x 24,
# and 16 x 32 with the longest z pencils); the widest columns (M = 128) run more
# workgroups than the fused pass has partial records
PLANE_SHAPES = [(4, 4, 4), (16, 16, 16), (6, 12, 8), (64, 16, 16), (8, 32, 8), (16, 4, 32), (24, 8, 24),
                (12, 6, 24), (256, 8, 8), (32, 4, 16), (8, 24, 6), (8, 24, 24), (6, 16, 32)]


def eifp():
    from paper_2210_06232_amd import eifp as m
    m.load()
    return m


def rounded32(F):
    return np.ascontiguousarray(np.asarray(F, dtype=np.float32).astype(np.float64))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", PLANE_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_plane_step_matches_oracle(shape, prec):
    m = eifp()
    H, E = inputs.white_noise_fields(shape, seed=400 + sum(shape))  # full spectrum, Nyquist included
    H, E = rounded32(H), rounded32(E)
    mu, eps, tau = 1.3, 0.8, 0.17
    Ho, Eo, _ = orc.step(H, E, DOMAIN, mu, eps, tau, 1)
    with m.Solver(H, E, DOMAIN, mu, eps, prec) as s:
        s.step(tau, 1)
        Hg, Eg = s.fields()
        got = s.invariants()
    en = energy_rel_error(Hg, Eg, Ho, Eo, mu, eps)
    el = elementwise_rel_error(Hg, Eg, Ho, Eo, mu, eps)
    print(f"{shape} {prec}: energy-norm {en:.3e}, element-wise {el:.3e}", flush=True)
    assert en <= TOL[prec] and el <= TOL[prec]
    # the invariants of the new state, summed by the plane pass and finalized by the x
    # kernel after it, against the oracle's physical-space values (as in the strided
    # passes' test: helicity and momentum against sqrt(E1 E2), the divergence norms
    # against their own size)
    want = orc.invariants(Ho, Eo, DOMAIN, mu, eps)
    tol = 1e-12 if prec == "fp64" else 1e-6
    e_ref = math.sqrt(want["E1"] * want["E2"])
    assert abs(got["energy"] - want["E1"]) <= tol * want["E1"]
    assert abs(got["helicity"] - want["H1"]) <= tol * e_ref
    for k, c in enumerate("xyz"):
        assert abs(got["momentum"][k] - want[f"M1_{c}"]) <= tol * e_ref
    dscale = max(1.0, want["divH_l2"], want["divE_l2"])
    assert abs(got["div_h_l2"] - want["divH_l2"]) <= tol * dscale * 10
    assert abs(got["div_e_l2"] - want["divE_l2"]) <= tol * dscale * 10


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(16, 16, 16), (32, 16, 16), (64, 8, 32)], ids=lambda s: "x".join(map(str, s)))
def test_plane_multi_step_call_equals_single_steps_bitwise(shape, prec):
    m = eifp()
    H, E = inputs.random_fields(shape, DOMAIN, workload=5, p=2.0)
    out = []
    for calls in ((6,), (1,) * 6, (4, 2)):
        with m.Solver(H, E, DOMAIN, 1.1, 0.9, prec) as s:
            for n in calls:
                s.step(0.13, n)
            out.append((s.fields(), s.invariants()))
    for (Hg, Eg), inv in out[1:]:
        np.testing.assert_array_equal(Hg, out[0][0][0])
        np.testing.assert_array_equal(Eg, out[0][0][1])
        assert {k: v for k, v in inv.items() if k != "t"} == {k: v for k, v in out[0][1].items() if k != "t"}


def test_plane_steps_invariants_agree_with_the_strided_evaluation():
    # the invariants a plane step reports, and those the strided forward passes compute
    # for the same state (eifp_invariants after reloading the fields), agree to round-off
    m = eifp()
    shape = (32, 16, 16)
    H, E = inputs.random_fields(shape, DOMAIN, workload=6, p=2.0)
    with m.Solver(H, E, DOMAIN, 1.0, 2.0, "fp64") as s:
        s.step(0.1, 3)
        inv_step = s.invariants()
        Hg, Eg = s.fields()
    with m.Solver(Hg, Eg, DOMAIN, 1.0, 2.0, "fp64") as s:
        inv_fresh = s.invariants()
    for k in ("energy", "helicity"):
        scale = max(abs(inv_fresh[k]), 1e-3 * abs(inv_fresh["energy"]))
        assert abs(inv_step[k] - inv_fresh[k]) <= 1e-13 * scale, (k, inv_step[k], inv_fresh[k])
