"""Pins of the oracle's force G = dL/dRe U + i dL/dIm U, L = Re<X, D[U] Y>.

The paper mentions the HMC (Sec. 2.1) whose fermion force this is, without
a formula.  Checks against mathematics:

* exact linearity: D is affine in U, so Re<X, (D[E] - D[0]) Y> equals
  sum Re tr(G^+ E) for ANY link field E (not only SU(2)) — this determines G
  completely given the pinned operator;
* the Euler identity sum Re tr(G^+ U) = Re<X, D Y> - m Re<X, Y>;
* autograd of an independent torch (roll-based) implementation of D;
* central finite differences (eps = 1e-6) of the fermion action
  S = phi^+ (D^+ D^)^{-1} phi at 4^4, with dense solves, against
  dS/dU = (2/m) G[X, Y].
"""
import numpy as np
import pytest
import torch

from oracle import dense
from paper_2411_18511_amd import inputs


def _links(dims, n, seed, oracle):
    Uf = inputs.gauge_field(dims, seed)
    return Uf if n == 2 else oracle.represent_adjoint(Uf).astype(np.complex128)


@pytest.mark.parametrize("n", [2, 3])
def test_exact_linearity(oracle, n):
    dims = (4, 2, 4, 2)
    rng = np.random.default_rng(5)
    X = inputs.gaussian_spinor(dims, n, 1)
    Y = inputs.gaussian_spinor(dims, n, 2)
    E = rng.standard_normal((4,) + dims + (n, n)) + 1j * rng.standard_normal((4,) + dims + (n, n))
    Z = np.zeros_like(E)
    m0 = -0.3
    lhs = np.real(oracle.inner(X, oracle.dirac(E, Y, m0) - oracle.dirac(Z, Y, m0)))
    G = oracle.force(X, Y)
    rhs = np.real(np.sum(np.conj(G) * E))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # single-link directions: each entry of G individually
    for _ in range(20):
        Ek = np.zeros_like(E)
        idx = tuple(rng.integers(0, s) for s in E.shape)
        val = complex(rng.standard_normal(), rng.standard_normal())
        Ek[idx] = val
        lhs = np.real(oracle.inner(X, oracle.dirac(Ek, Y, m0) - oracle.dirac(Z, Y, m0)))
        assert abs(lhs - np.real(np.conj(G[idx]) * val)) < 1e-12


@pytest.mark.parametrize("n", [2, 3])
def test_euler_identity(oracle, n):
    dims = (4, 4, 2, 4)
    m0 = -0.4
    U = _links(dims, n, 7, oracle)
    X = inputs.gaussian_spinor(dims, n, 8)
    Y = inputs.gaussian_spinor(dims, n, 9)
    G = oracle.force(X, Y)
    lhs = np.real(np.sum(np.conj(G) * U))
    rhs = np.real(oracle.inner(X, oracle.dirac(U, Y, m0))) - (4 + m0) * np.real(oracle.inner(X, Y))
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)


def _torch_dirac(U, psi, m0, g):
    """Independent roll-based D for the autograd check (torch, CPU, complex128)."""
    T = U.shape[1]
    out = (4 + m0) * psi
    tsign = torch.ones(U.shape[1:5], dtype=torch.float64)
    tsign[T - 1] = -1.0  # s_0(x) = -1 at t = T-1
    for mu in range(4):
        s = tsign if mu == 0 else torch.ones_like(tsign)
        fwd = torch.roll(psi, -1, dims=mu)  # psi(x + mu)
        Ufwd = torch.einsum("...ij,...aj->...ai", U[mu], fwd)
        term = Ufwd - torch.einsum("ab,...bi->...ai", g[mu], Ufwd)
        out = out - 0.5 * s[..., None, None] * term
        Ud = torch.conj(U[mu]).transpose(-1, -2)
        bwd = torch.einsum("...ij,...aj->...ai", Ud, psi)  # U(x)^+ psi(x), then shift to x + mu
        bwd = bwd + torch.einsum("ab,...bi->...ai", g[mu], bwd)
        bwd = (s[..., None, None] * bwd)
        out = out - 0.5 * torch.roll(bwd, 1, dims=mu)
    return out


@pytest.mark.parametrize("n", [2, 3])
def test_autograd_of_independent_torch_operator(oracle, n):
    dims = (4, 2, 2, 4)
    m0 = -0.1
    U = _links(dims, n, 13, oracle)
    X = inputs.gaussian_spinor(dims, n, 14)
    Y = inputs.gaussian_spinor(dims, n, 15)
    g = [torch.tensor(oracle.gamma(m)) for m in range(4)]
    Ut = torch.tensor(U, requires_grad=True)
    Dy = _torch_dirac(Ut, torch.tensor(Y), m0, g)
    # the torch operator itself agrees with the oracle
    assert np.abs(Dy.detach().numpy() - oracle.dirac(U, Y, m0)).max() < 1e-13
    L = torch.real(torch.sum(torch.conj(torch.tensor(X)) * Dy))
    L.backward()
    G = oracle.force(X, Y)
    assert np.abs(Ut.grad.numpy() - G).max() < 1e-13
    if n == 3:
        Gr = oracle.force(X, Y, real_links=True)
        Ur = torch.tensor(U.real, requires_grad=True)
        Dy = _torch_dirac(Ur.to(torch.complex128), torch.tensor(Y), m0, g)
        L = torch.real(torch.sum(torch.conj(torch.tensor(X)) * Dy))
        L.backward()
        assert np.abs(Ur.grad.numpy() - Gr).max() < 1e-13


def _dense_action(U, phi_e_vec, m0, dims, n):
    D = dense.dirac_matrix(U, m0)
    Dee, Deo, Doe, Doo = dense.schur_blocks(D, dims, n)
    Dh = Dee - Deo @ Doe / (4 + m0)
    y = np.linalg.solve(Dh.conj().T, phi_e_vec)
    return float(np.real(np.vdot(y, y)))


@pytest.mark.slow
@pytest.mark.parametrize("n", [2, 3])
def test_action_force_central_differences(oracle, n):
    """dS/dU = (2/m) G[X, Y] against central differences with eps = 1e-6 at 4^4."""
    dims = (4, 4, 4, 4)
    m0 = -0.4
    U = _links(dims, n, 17, oracle)
    phi = oracle.restrict(inputs.gaussian_spinor(dims, n, 18), 0)
    e, _ = dense.parity_index(dims, n)
    phi_vec = phi.ravel()[e]
    F, xi, info = oracle.action_force(U, phi, m0, tol=1e-13, real_links=(n == 3))
    rng = np.random.default_rng(19)
    eps = 1e-6
    directions = []
    for _ in range(6):
        E = rng.standard_normal(U.shape)
        if n == 2:
            E = E + 1j * rng.standard_normal(U.shape)
        directions.append(E)
    for _ in range(10):
        E = np.zeros(U.shape, np.complex128 if n == 2 else np.float64)
        idx = tuple(rng.integers(0, s) for s in U.shape)
        E[idx] = 1.0 if (n == 3 or rng.random() < 0.5) else 1j
        directions.append(E)
    for E in directions:
        sp = _dense_action(U + eps * E, phi_vec, m0, dims, n)
        sm = _dense_action(U - eps * E, phi_vec, m0, dims, n)
        fd = (sp - sm) / (2 * eps)
        an = float(np.real(np.sum(np.conj(F) * E)))
        scale = max(abs(an), 1e-3 * np.abs(F).max())
        assert abs(fd - an) <= 1e-6 * scale + 1e-7, (fd, an)
