"""Pins of the oracle's clover term (the paper's Sec. 2.2 diagonal term; the
paper gives no formula, the reading is stated in oracle/oracle.c).

* free field: A = 0;
* A is Hermitian and commutes with g5 (block diagonal in chirality);
* closed form for a constant abelian field U_1(x) = exp(i phi x2 s3),
  phi = 2 pi k / L2: every (1,2) plaquette equals exp(-i phi s3), so
  F_12 = -i sin(phi) s3 and, with sigma_12 = -diag(s3, s3) in the chiral
  basis, A = -(c_sw / 2) sin(phi) s3(spin) (x) s3(colour), all other planes 0
  — pins the leaf orientation, the 1/8 and the i/4;
* gauge covariance A[U^g](x) = g(x) A[U](x) g(x)^+ and of D_sw;
* an independent dense D_sw: the Schur complement equals the even/odd
  operator M_ee - D_eo M_oo^-1 D_oe, determinants factorise, CG solves it;
* the exponentiated clover M = m exp(A/m): the matrix exponential agrees
  with scipy's Pade-based expm and with its power series, M vanishes to
  m at c_sw = 0, equals m exp(diag/m) for the abelian field, agrees with
  m + A + A^2/(2m) to third order in c_sw, and M^{-1} = exp(-A/m)/m.
"""
import numpy as np
import pytest

from oracle import dense
from paper_2411_18511_amd import inputs


def _links(dims, n, seed, oracle, kind="haar"):
    Uf = inputs.gauge_field(dims, seed, kind=kind)
    return Uf if n == 2 else oracle.represent_adjoint(Uf).astype(np.complex128)


def test_free_field_clover_vanishes(oracle):
    dims = (4, 4, 2, 2)
    for n in (2, 3):
        U = np.zeros((4,) + dims + (n, n), np.complex128)
        for i in range(n):
            U[..., i, i] = 1
        assert np.abs(oracle.clover(U, 1.7)).max() < 1e-15


@pytest.mark.parametrize("n", [2, 3])
def test_clover_hermitian_chiral(oracle, n):
    U = _links((4, 2, 4, 2), n, 3, oracle)
    A = oracle.clover(U, 1.3)
    assert np.abs(A - np.conj(np.swapaxes(A, -1, -2))).max() < 1e-14
    g5 = np.kron(oracle.gamma5(), np.eye(n))
    assert np.abs(A @ g5 - g5 @ A).max() < 1e-14
    assert np.abs(A[..., : 2 * n, 2 * n:]).max() < 1e-14
    assert np.abs(A).max() > 0.1


def test_abelian_constant_field_closed_form(oracle):
    dims = (2, 4, 6, 2)
    k = 1
    phi = 2 * np.pi * k / dims[2]
    csw = 1.9
    U = np.zeros((4,) + dims + (2, 2), np.complex128)
    U[..., 0, 0] = 1
    U[..., 1, 1] = 1
    x2 = np.arange(dims[2]).reshape(1, 1, -1, 1)
    U[1, ..., 0, 0] = np.exp(1j * phi * x2)
    U[1, ..., 1, 1] = np.exp(-1j * phi * x2)
    A = oracle.clover(U, csw)
    s3_spin = np.array([1, -1, 1, -1])
    s3_col = np.array([1, -1])
    want = np.diag(-(csw / 2) * np.sin(phi) * np.kron(s3_spin, s3_col)).astype(np.complex128)
    assert np.abs(A - want).max() < 1e-14
    # and D_sw adds exactly that diagonal to D
    psi = inputs.gaussian_spinor(dims, 2, 5)
    diff = oracle.dirac_clover(U, psi, -0.3, csw) - oracle.dirac(U, psi, -0.3)
    assert np.abs(diff - oracle.apply_site_matrix(np.broadcast_to(want, A.shape), psi)).max() < 1e-13


@pytest.mark.parametrize("n", [2, 3])
def test_clover_gauge_covariance(oracle, n):
    dims = (4, 2, 4, 2)
    rng = inputs.rng_for(7)
    Uf = inputs.gauge_field(dims, 8)
    g = inputs.gauge_transform(rng, dims)
    Ug = np.empty_like(Uf)
    for mu in range(4):
        Ug[mu] = g @ Uf[mu] @ np.conj(np.swapaxes(np.roll(g, -1, axis=mu), -1, -2))
    if n == 2:
        U, Ut, gR = Uf, Ug, g
    else:
        U = oracle.represent_adjoint(Uf).astype(np.complex128)
        Ut = oracle.represent_adjoint(Ug).astype(np.complex128)
        gR = oracle.represent_adjoint(g).astype(np.complex128)
    G = np.einsum("ab,...ij->...aibj", np.eye(4), gR).reshape(gR.shape[:-2] + (4 * n, 4 * n))
    A = oracle.clover(U, 1.1)
    At = oracle.clover(Ut, 1.1)
    assert np.abs(At - G @ A @ np.conj(np.swapaxes(G, -1, -2))).max() < 1e-13
    psi = inputs.gaussian_spinor(dims, n, 9)
    gpsi = np.einsum("...ij,...aj->...ai", gR, psi)
    lhs = oracle.dirac_clover(Ut, gpsi, -0.2, 1.1)
    rhs = np.einsum("...ij,...aj->...ai", gR, oracle.dirac_clover(U, psi, -0.2, 1.1))
    assert np.abs(lhs - rhs).max() < 1e-12


@pytest.mark.parametrize("kind", ["sw", "exp"])
@pytest.mark.parametrize("dims,n", [((2, 2, 2, 2), 2), ((4, 2, 2, 2), 2), ((2, 2, 2, 2), 3)])
def test_clover_dense_schur(oracle, dims, n, kind):
    m0, csw = -0.3, 1.2
    m = 4.0 + m0
    U = _links(dims, n, 11, oracle)
    D = dense.dirac_matrix(U, m0)
    M, _ = oracle.clover_diag(U, m0, csw, kind)
    A = M.reshape(-1, 4 * n, 4 * n) - m * np.eye(4 * n)
    blk = 4 * n
    for s in range(A.shape[0]):
        D[s * blk:(s + 1) * blk, s * blk:(s + 1) * blk] += A[s]
    psi = inputs.gaussian_spinor(dims, n, 12)
    assert np.abs(oracle.dirac_clover(U, psi, m0, csw, kind).ravel() - D @ psi.ravel()).max() < 1e-13
    Dee, Deo, Doe, Doo = dense.schur_blocks(D, dims, n)
    S = Dee - Deo @ np.linalg.solve(Doo, Doe)
    e, _ = dense.parity_index(dims, n)
    shape = tuple(dims) + (4, n)
    cols = np.empty((len(e), len(e)), np.complex128)
    for k in range(len(e)):
        v = np.zeros(int(np.prod(shape)), np.complex128)
        v[e[k]] = 1
        cols[:, k] = oracle.dhat_clover(U, v.reshape(shape), m0, csw, kind=kind).ravel()[e]
    assert np.abs(cols - S).max() < 1e-13
    _, ld = np.linalg.slogdet(D)
    _, lh = np.linalg.slogdet(S)
    _, lo = np.linalg.slogdet(Doo)
    assert abs(ld - (lh + lo)) < 1e-10
    # g5-hermiticity of the clover D^
    phe = oracle.restrict(inputs.gaussian_spinor(dims, n, 13), 0)
    pse = oracle.restrict(psi, 0)
    lhs = oracle.inner(phe, oracle.dhat_clover(U, pse, m0, csw, kind=kind))
    rhs = oracle.inner(oracle.dhat_clover_dagger(U, phe, m0, csw, kind=kind), pse)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("kind", ["sw", "exp"])
def test_clover_cg(oracle, kind):
    dims, n, m0, csw = (4, 4, 2, 4), 2, -0.2, 1.0
    U = _links(dims, n, 21, oracle, kind="smeared")
    b = oracle.restrict(inputs.gaussian_spinor(dims, n, 22), 0)
    x, info = oracle.cg_clover(U, b, m0, csw, tol=1e-11, kind=kind)
    assert info["true_rel_residual"] <= 1e-11
    assert oracle.true_residual_clover(U, b, x, m0, csw, kind=kind) <= 1e-11


def test_expm_hermitian_pins(oracle):
    import scipy.linalg

    rng = np.random.default_rng(5)
    for n in (4, 6):
        Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        X = (Z + Z.conj().T) / 4
        E = oracle.expm_hermitian(X)
        assert np.abs(E - scipy.linalg.expm(X)).max() < 1e-13 * np.abs(E).max()
        # power series, summed until the terms vanish
        S, T = np.eye(n, dtype=complex), np.eye(n, dtype=complex)
        for k in range(1, 60):
            T = T @ X / k
            S = S + T
        assert np.abs(E - S).max() < 1e-13 * np.abs(E).max()
        assert np.abs(E @ oracle.expm_hermitian(-X) - np.eye(n)).max() < 1e-13
    d = np.array([0.3, -1.2, 2.0])
    assert np.abs(oracle.expm_hermitian(np.diag(d)) - np.diag(np.exp(d))).max() < 1e-15 * np.exp(2.0)


def test_exp_clover_special_cases(oracle):
    m0 = -0.3
    m = 4.0 + m0
    # c_sw = 0: M = m, M^{-1} = 1/m
    U = _links((4, 2, 2, 2), 2, 3, oracle)
    M, Mi = oracle.clover_diag(U, m0, 0.0, "exp")
    assert np.abs(M - m * np.eye(8)).max() < 1e-14 and np.abs(Mi - np.eye(8) / m).max() < 1e-15
    # abelian constant field: A is diagonal, so M = m exp(diag(A)/m) elementwise
    dims, k, csw = (2, 4, 6, 2), 1, 1.9
    phi = 2 * np.pi * k / dims[2]
    U = np.zeros((4,) + dims + (2, 2), np.complex128)
    U[..., 0, 0] = 1
    U[..., 1, 1] = 1
    x2 = np.arange(dims[2]).reshape(1, 1, -1, 1)
    U[1, ..., 0, 0] = np.exp(1j * phi * x2)
    U[1, ..., 1, 1] = np.exp(-1j * phi * x2)
    a = -(csw / 2) * np.sin(phi) * np.kron([1, -1, 1, -1], [1, -1])
    M, Mi = oracle.clover_diag(U, m0, csw, "exp")
    assert np.abs(M - np.diag(m * np.exp(a / m))).max() < 1e-14
    assert np.abs(Mi - np.diag(np.exp(-a / m) / m)).max() < 1e-15
    # small c_sw: m exp(A/m) = m + A + A^2/(2m) + O(c_sw^3)
    U = _links((4, 2, 2, 2), 3, 9, oracle)
    errs = []
    for c in (0.02, 0.04):
        A = oracle.clover(U, c)
        M, Mi = oracle.clover_diag(U, m0, c, "exp")
        errs.append(np.abs(M - m * np.eye(12) - A - A @ A / (2 * m)).max())
        assert np.abs(M @ Mi - np.eye(12)).max() < 1e-14
    assert 6.0 < errs[1] / errs[0] < 10.0  # third order


def test_exp_clover_covariance(oracle):
    dims = (4, 2, 4, 2)
    rng = inputs.rng_for(7)
    Uf = inputs.gauge_field(dims, 8)
    g = inputs.gauge_transform(rng, dims)
    Ug = np.empty_like(Uf)
    for mu in range(4):
        Ug[mu] = g @ Uf[mu] @ np.conj(np.swapaxes(np.roll(g, -1, axis=mu), -1, -2))
    G = np.einsum("ab,...ij->...aibj", np.eye(4), g).reshape(g.shape[:-2] + (8, 8))
    M, _ = oracle.clover_diag(Uf, -0.2, 1.3, "exp")
    Mt, _ = oracle.clover_diag(Ug, -0.2, 1.3, "exp")
    assert np.abs(Mt - G @ M @ np.conj(np.swapaxes(G, -1, -2))).max() < 1e-13
