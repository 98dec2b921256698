"""Pins of the oracle's mode-wise propagator (Prop. 2.1/2.2, Alg. 2 steps 2-4).

The closed-form coefficients are checked against the matrix exponential of the
spectral Maxwell generator written from (1.1) (curl -> i b x), and against the
structural facts that follow from it: unitarity in the (sqrt(mu) H, sqrt(eps) E)
variables, the identity at t = 0 and at b = 0, the group property, time reversal,
and conservation of the longitudinal parts b.H^, b.E^ (Thm 4.6)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as orc


def cross_matrix(b):
    bx, by, bz = b
    return np.array([[0.0, -bz, by], [bz, 0.0, -bx], [-by, bx, 0.0]])


def generator(b, mu, eps):
    # d/dt H^ = -(1/mu) (i b) x E^,  d/dt E^ = (1/eps) (i b) x H^   -- (1.1) in Fourier space
    K = 1j * cross_matrix(b)
    G = np.zeros((6, 6), complex)
    G[:3, 3:] = -K / mu
    G[3:, :3] = K / eps
    return G


CASES = [
    ((1.0, 2.0, -3.0), 0.37, 1.0, 1.0),
    ((0.5, 0.0, 0.0), 2.0, 1.0, 2.0),
    ((3.0, -1.0, 4.0), 10.0, 2.0, 0.5),
    ((0.0, 0.0, 1e-5), 0.1, 1.3, 0.7),       # tiny phase: r1, r2 near their limits
    ((12.0, 7.0, -30.0), 5.0, 1.0, 1.5),     # large phase, many turns
    ((1.0, 1.0, 1.0), -0.8, 1.0, 1.0),       # negative time
]


@pytest.mark.parametrize("b,t,mu,eps", CASES)
def test_closed_form_equals_matrix_exponential(b, t, mu, eps):
    P = orc.propagator(b, t, mu, eps)
    want = scipy.linalg.expm(t * generator(np.array(b), mu, eps))
    np.testing.assert_allclose(P, want, atol=2e-13 * max(1.0, np.abs(want).max()))


@pytest.mark.parametrize("b,t,mu,eps", CASES)
def test_scaled_map_is_unitary(b, t, mu, eps):
    P = orc.propagator(b, t, mu, eps)
    S = np.diag([np.sqrt(mu)] * 3 + [np.sqrt(eps)] * 3)
    U = S @ P @ np.linalg.inv(S)
    np.testing.assert_allclose(U @ U.conj().T, np.eye(6), atol=1e-13)


def test_identity_cases():
    np.testing.assert_allclose(orc.propagator((1.0, -2.0, 0.5), 0.0, 1.3, 0.4), np.eye(6), atol=0)
    np.testing.assert_allclose(orc.propagator((0.0, 0.0, 0.0), 3.0, 1.3, 0.4), np.eye(6), atol=0)
    c, s = orc.coefficients((0.0, 0.0, 0.0), 5.0)
    np.testing.assert_allclose(c, [1, 0, 0, 1, 0, 1], atol=0)
    np.testing.assert_allclose(s, [0, 0, 0], atol=0)


def test_group_property_and_reversal():
    b, mu, eps = (1.5, -0.5, 2.0), 1.2, 0.8
    P1 = orc.propagator(b, 0.3, mu, eps)
    P2 = orc.propagator(b, 1.1, mu, eps)
    np.testing.assert_allclose(P1 @ P2, orc.propagator(b, 1.4, mu, eps), atol=1e-14)
    np.testing.assert_allclose(orc.propagator(b, -0.3, mu, eps) @ P1, np.eye(6), atol=1e-14)


def test_longitudinal_parts_are_held():
    # Thm 4.6 (with the printed identities read as b^T C = b^T, b^T S = 0)
    b = np.array([0.7, -2.0, 1.3])
    P = orc.propagator(b, 2.5, 1.0, 3.0)
    L = np.zeros((2, 6))
    L[0, :3] = b
    L[1, 3:] = b
    np.testing.assert_allclose(L @ P, L, atol=1e-14)


def test_coefficient_symmetry_in_b():
    # c_ij are even in b, s_ij odd: a real field keeps a Hermitian spectrum.
    b = np.array([0.3, 1.7, -2.2])
    c1, s1 = orc.coefficients(b, 0.9)
    c2, s2 = orc.coefficients(-b, 0.9)
    np.testing.assert_allclose(c1, c2, atol=0)
    np.testing.assert_allclose(s1, -s2, atol=0)
