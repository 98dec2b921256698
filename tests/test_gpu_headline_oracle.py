"""The 256^3 workload the benchmark times (box [0, 2pi] x [0, 4pi] x [0, 2pi], mu = eps = 1,
tau = 0.1, the seeded transverse fields with spectrum (1 + |k|^2)^-2): one FP64 step on the
GPU, in the launch configuration the benchmark uses, against one oracle step over the
whole grid (Def. 2.3 / Alg. 2) at 1e-12, in the energy norm and element by element.  One
oracle step at this size takes about half a minute to a minute on one host core."""
import time

import pytest

from oracle import oracle as orc
from paper_2210_06232_amd.workload import HEADLINE, headline_inputs
from tests.helpers import elementwise_rel_error, energy_rel_error

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def test_headline_256_fp64_one_step_vs_oracle():
    from paper_2210_06232_amd import eifp
    eifp.load()
    H, E = headline_inputs()
    dom = tuple(HEADLINE["domain"])
    mu, eps, tau = HEADLINE["mu"], HEADLINE["eps"], HEADLINE["tau"]
    with eifp.Solver(H, E, dom, mu, eps, "fp64") as s:
        s.step(tau, 1)
        Hg, Eg = s.fields()
    t0 = time.perf_counter()
    Ho, Eo, _ = orc.step(H, E, dom, mu, eps, tau, 1)
    en = energy_rel_error(Hg, Eg, Ho, Eo, mu, eps)
    el = elementwise_rel_error(Hg, Eg, Ho, Eo, mu, eps)
    print(f"256^3 headline fp64, one step: energy-norm {en:.3e}, element-wise {el:.3e} "
          f"(oracle {time.perf_counter() - t0:.1f} s)", flush=True)
    assert en <= FP64_TOL and el <= FP64_TOL
