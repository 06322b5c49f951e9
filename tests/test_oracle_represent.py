"""Pins of the oracle's adjoint map R_ab(U) = tr(s_a U s_b U^+) / 2.

The paper (Sec. 1) runs fermions in higher representations of SU(N); for
SU(2) the adjoint is the 3-dimensional real representation.  Checks against
mathematics: R is real orthogonal with det 1, a group homomorphism, its trace
is the adjoint character |tr U|^2 - 1, and for U = exp(i theta n.s / 2) it is
the closed-form (Rodrigues) rotation by -theta about n.
"""
import numpy as np

from paper_2411_18511_amd import inputs


def test_orthogonal_det_one(oracle):
    U = inputs.haar_su2(inputs.rng_for(1), (500,))
    R = oracle.represent_adjoint(U)
    assert R.dtype == np.float64
    eye = np.einsum("lab,lcb->lac", R, R)
    assert np.abs(eye - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(R) - 1).max() < 1e-14


def test_homomorphism(oracle):
    rng = inputs.rng_for(2)
    A = inputs.haar_su2(rng, (200,))
    B = inputs.haar_su2(rng, (200,))
    lhs = oracle.represent_adjoint(A @ B)
    rhs = oracle.represent_adjoint(A) @ oracle.represent_adjoint(B)
    assert np.abs(lhs - rhs).max() < 1e-14
    # inverse maps to transpose
    Ad = np.conj(np.swapaxes(A, -1, -2))
    assert np.abs(oracle.represent_adjoint(Ad) - np.swapaxes(oracle.represent_adjoint(A), -1, -2)).max() < 1e-14


def test_adjoint_character(oracle):
    U = inputs.haar_su2(inputs.rng_for(3), (300,))
    R = oracle.represent_adjoint(U)
    trU = np.trace(U, axis1=-2, axis2=-1)
    assert np.abs(np.trace(R, axis1=-2, axis2=-1) - (np.abs(trU) ** 2 - 1)).max() < 1e-14


def test_rodrigues_closed_form(oracle):
    rng = np.random.default_rng(4)
    pauli = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
    for _ in range(50):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        th = rng.uniform(-np.pi, np.pi)
        U = np.cos(th / 2) * np.eye(2) + 1j * np.sin(th / 2) * sum(n[k] * pauli[k] for k in range(3))
        K = np.array([[0, -n[2], n[1]], [n[2], 0, -n[0]], [-n[1], n[0], 0]])
        # rotation by -theta about n
        want = np.cos(th) * np.eye(3) - np.sin(th) * K + (1 - np.cos(th)) * np.outer(n, n)
        got = oracle.represent_adjoint(U[None])[0]
        assert np.abs(got - want).max() < 1e-14


def test_identity_and_centre(oracle):
    U = np.stack([np.eye(2), -np.eye(2)]).astype(np.complex128)
    R = oracle.represent_adjoint(U)
    assert np.array_equal(R[0], np.eye(3))
    assert np.array_equal(R[1], np.eye(3))
