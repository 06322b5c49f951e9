"""Pins of the oracle's Wilson-Dirac operator against mathematics, not against itself.

The paper (Sec. 2.1, Table 1) names the unimproved Wilson-Dirac operator and
its even/odd preconditioned form but prints no formula or worked example, so
every check here is a closed form or an invariant that a dropped term, a
wrong sign, a swapped U/U^+ or a wrong neighbour index would break:

* Clifford algebra of the gamma basis; g5 diagonal in the chiral basis;
* free field (U = 1): plane waves are eigenvectors with the closed-form
  momentum-space matrix m0 + sum(1 - cos p) + i sum g_mu sin p_mu, with
  antiperiodic time momenta — catches sign, factor 1/2, neighbour and
  boundary mistakes;
* free-field spectrum of the dense matrix equals the closed form (multiset);
* g5-hermiticity and gauge covariance for random links — catch U/U^+ swaps,
  wrong link sites and projector signs that the free field cannot see;
* the loop oracle equals an independently assembled dense matrix;
* Schur-complement identities for the even/odd operator.
"""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

from oracle import dense
from paper_2411_18511_amd import inputs


def _unit_links(dims, n):
    U = np.zeros((4,) + tuple(dims) + (n, n), np.complex128)
    for i in range(n):
        U[..., i, i] = 1
    return U


def _field(dims, n, seed):
    return inputs.gaussian_spinor(dims, n, seed)


def _links(dims, n, seed, oracle):
    Uf = inputs.gauge_field(dims, seed)
    if n == 2:
        return Uf
    return oracle.represent_adjoint(Uf).astype(np.complex128)


def test_clifford_algebra(oracle):
    g = [oracle.gamma(m) for m in range(4)]
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            anti = g[a] @ g[b] + g[b] @ g[a]
            assert np.allclose(anti, 2 * (a == b) * np.eye(4))
    g5 = oracle.gamma5()
    assert np.allclose(g5, np.diag([-1, -1, 1, 1]))
    for a in range(4):
        assert np.allclose(g5 @ g[a], -g[a] @ g5)
    # the dense builder constructs its own basis; both must agree
    for a, b in zip(g, dense.gammas()):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 2, 8), (4, 6, 4, 2)])
@pytest.mark.parametrize("n", [2, 3])
def test_free_field_plane_waves(oracle, dims, n):
    """D e^{ipx} u = [m0 + sum(1 - cos p) + i sum g_mu sin p_mu] u e^{ipx}."""
    m0 = -0.37
    rng = np.random.default_rng(7)
    g = [oracle.gamma(m) for m in range(4)]
    U = _unit_links(dims, n)
    coords = np.meshgrid(*[np.arange(L) for L in dims], indexing="ij")
    for _ in range(4):
        nn = [rng.integers(0, L) for L in dims]
        p = [(2 * np.pi * nn[0] + np.pi) / dims[0]] + [2 * np.pi * nn[k] / dims[k] for k in (1, 2, 3)]
        u = rng.standard_normal((4, n)) + 1j * rng.standard_normal((4, n))
        phase = np.exp(1j * sum(p[m] * coords[m] for m in range(4)))
        psi = phase[..., None, None] * u
        Dp = (m0 + sum(1 - np.cos(q) for q in p)) * np.eye(4) + 1j * sum(
            g[m] * np.sin(p[m]) for m in range(4))
        want = phase[..., None, None] * (Dp @ u)
        got = oracle.dirac(U, psi, m0)
        assert np.abs(got - want).max() < 1e-12


def _multiset_close(a, b):
    cost = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(cost)
    return cost[r, c].max()


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 2)])
def test_free_field_spectrum_dense(oracle, dims):
    m0 = -0.2
    n = 2
    U = _unit_links(dims, n)
    D = dense.dirac_matrix(U, m0)
    ev = np.linalg.eigvals(D)
    want = dense.free_spectrum(dims, m0, n)
    assert len(ev) == len(want)
    assert _multiset_close(ev, want) < 1e-10
    # the loop oracle applies the same matrix
    psi = _field(dims, n, 3)
    assert np.abs(oracle.dirac(U, psi, m0).ravel() - D @ psi.ravel()).max() < 1e-13


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 2), (2, 4, 2, 2)])
@pytest.mark.parametrize("n", [2, 3])
def test_oracle_equals_dense_matrix(oracle, dims, n):
    U = _links(dims, n, 11, oracle)
    psi = _field(dims, n, 12)
    D = dense.dirac_matrix(U, -0.5)
    got = oracle.dirac(U, psi, -0.5).ravel()
    assert np.abs(got - D @ psi.ravel()).max() < 1e-13


@pytest.mark.parametrize("n", [2, 3])
def test_gamma5_hermiticity(oracle, n):
    dims = (4, 4, 2, 6)
    m0 = -0.4
    U = _links(dims, n, 21, oracle)
    phi = _field(dims, n, 22)
    psi = _field(dims, n, 23)
    lhs = oracle.inner(phi, oracle.dirac(U, psi, m0))
    rhs = oracle.inner(oracle.dirac_dagger(U, phi, m0), psi)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    # even/odd operator
    phe = oracle.restrict(phi, 0)
    pse = oracle.restrict(psi, 0)
    lhs = oracle.inner(phe, oracle.dhat(U, pse, m0))
    rhs = oracle.inner(oracle.dhat_dagger(U, phe, m0), pse)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_gamma5_hermiticity_dense(oracle):
    dims = (2, 2, 2, 2)
    U = _links(dims, 2, 31, oracle)
    D = dense.dirac_matrix(U, -0.1)
    V = 16
    G5 = np.kron(np.eye(V), np.kron(oracle.gamma5(), np.eye(2)))
    assert np.abs(D.conj().T - G5 @ D @ G5).max() < 1e-14


@pytest.mark.parametrize("n", [2, 3])
def test_gauge_covariance(oracle, n):
    """D[U^g](g psi) = g D[U] psi with U^g_mu(x) = g(x) U_mu(x) g(x+mu)^+."""
    dims = (4, 2, 4, 6)
    m0 = -0.3
    rng = inputs.rng_for(41)
    Uf = inputs.gauge_field(dims, 42)
    g = inputs.gauge_transform(rng, dims)
    Ug = np.empty_like(Uf)
    for mu in range(4):
        g_fwd = np.roll(g, -1, axis=mu)
        Ug[mu] = g @ Uf[mu] @ np.conj(np.swapaxes(g_fwd, -1, -2))
    if n == 2:
        U, Ut, gR = Uf, Ug, g
    else:
        U = oracle.represent_adjoint(Uf).astype(np.complex128)
        Ut = oracle.represent_adjoint(Ug).astype(np.complex128)
        gR = oracle.represent_adjoint(g).astype(np.complex128)
    psi = _field(dims, n, 43)
    gpsi = np.einsum("...ij,...aj->...ai", gR, psi)
    lhs = oracle.dirac(Ut, gpsi, m0)
    rhs = np.einsum("...ij,...aj->...ai", gR, oracle.dirac(U, psi, m0))
    assert np.abs(lhs - rhs).max() < 1e-12
    # a field that is not a gauge transform of U gives a different result
    assert np.abs(oracle.dirac(U, gpsi, m0) - rhs).max() > 1e-3


@pytest.mark.parametrize("dims,n", [((2, 2, 2, 2), 2), ((4, 2, 2, 2), 2), ((2, 2, 2, 2), 3)])
def test_schur_complement(oracle, dims, n):
    """D^ equals the Schur complement of the dense D, and the determinants factor."""
    m0 = -0.25
    m = 4 + m0
    U = _links(dims, n, 51, oracle)
    D = dense.dirac_matrix(U, m0)
    Dee, Deo, Doe, Doo = dense.schur_blocks(D, dims, n)
    assert np.abs(Dee - m * np.eye(len(Dee))).max() < 1e-15
    assert np.abs(Doo - m * np.eye(len(Doo))).max() < 1e-15
    S = Dee - Deo @ np.linalg.solve(Doo, Doe)
    e, _ = dense.parity_index(dims, n)
    # D^ from the oracle, column by column
    ne = len(e)
    cols = np.empty((ne, ne), np.complex128)
    shape = tuple(dims) + (4, n)
    for k in range(ne):
        v = np.zeros(int(np.prod(shape)), np.complex128)
        v[e[k]] = 1
        cols[:, k] = oracle.dhat(U, v.reshape(shape), m0).ravel()[e]
    assert np.abs(cols - S).max() < 1e-13
    sd, ld = np.linalg.slogdet(D)
    sh, lh = np.linalg.slogdet(S)
    nodd = len(D) - ne
    assert abs(ld - (lh + nodd * np.log(m))) < 1e-10
    assert abs(sd - sh) < 1e-10


def test_even_odd_solve_equals_full_solve(oracle):
    dims = (4, 2, 2, 2)
    n = 2
    m0 = -0.2
    m = 4 + m0
    U = _links(dims, n, 61, oracle)
    b = _field(dims, n, 62)
    x_full = np.linalg.solve(dense.dirac_matrix(U, m0), b.ravel()).reshape(b.shape)
    be = oracle.restrict(b, 0)
    bo = oracle.restrict(b, 1)
    rhs_e = be - oracle.hop_block(U, bo, 0) / m
    # solve D^ x_e = rhs_e via the normal equations with the oracle CG
    xe, info = oracle.cg(U, oracle.dhat_dagger(U, rhs_e, m0), m0, tol=1e-13)
    xo = (bo - oracle.hop_block(U, xe, 1)) / m
    assert np.abs(xe + xo - x_full).max() < 1e-10


def test_hop_block_dagger_dense(oracle):
    dims = (2, 2, 2, 2)
    n = 2
    U = _links(dims, n, 71, oracle)
    D = dense.dirac_matrix(U, 0.0)
    _, Deo, Doe, _ = dense.schur_blocks(D, dims, n)
    e, o = dense.parity_index(dims, n)
    shape = tuple(dims) + (4, n)
    rng = np.random.default_rng(3)
    v = np.zeros(int(np.prod(shape)), np.complex128)
    v[e] = rng.standard_normal(len(e)) + 1j * rng.standard_normal(len(e))
    got = oracle.hop_block_dagger(U, v.reshape(shape), 1).ravel()
    assert np.abs(got[o] - Deo.conj().T @ v[e]).max() < 1e-14
    assert np.abs(got[e]).max() == 0
    got2 = oracle.hop_block(U, v.reshape(shape), 1).ravel()
    assert np.abs(got2[o] - Doe @ v[e]).max() < 1e-14


@pytest.mark.parametrize("n", [2, 3])
def test_normal_operator_hermitian_positive(oracle, n):
    dims = (4, 4, 2, 2)
    U = _links(dims, n, 81, oracle)
    u = oracle.restrict(_field(dims, n, 82), 0)
    v = oracle.restrict(_field(dims, n, 83), 0)
    m0 = -0.5
    a = oracle.inner(u, oracle.normal_op(U, v, m0))
    b = oracle.inner(oracle.normal_op(U, u, m0), v)
    assert abs(a - b) < 1e-11 * abs(a)
    assert np.real(oracle.inner(v, oracle.normal_op(U, v, m0))) > 0


@pytest.mark.parametrize("n", [2, 3])
def test_cg_matches_dense_solve(oracle, n):
    dims = (4, 4, 4, 4) if n == 2 else (4, 4, 2, 4)
    m0 = -0.2
    U = _links(dims, n, 91, oracle)
    b = oracle.restrict(_field(dims, n, 92), 0)
    x, info = oracle.cg(U, b, m0, tol=1e-10)
    assert info["true_rel_residual"] <= 1e-10
    assert oracle.true_residual(U, b, x, m0) <= 1e-10
    D = dense.dirac_matrix(U, m0)
    Dee, Deo, Doe, Doo = dense.schur_blocks(D, dims, n)
    S = Dee - Deo @ Doe / (4 + m0)
    e, _ = dense.parity_index(dims, n)
    xd = np.linalg.solve(S.conj().T @ S, b.ravel()[e])
    assert np.linalg.norm(x.ravel()[e] - xd) / np.linalg.norm(xd) < 1e-8


@pytest.mark.parametrize("n", [2, 3])
def test_native_cg_matches_dense_solve(oracle, n):
    """The C iteration of the oracle CG (used on the large lattices) solves the
    dense even/odd system, takes the same iterations as the numpy one, and its
    true residual routine equals the numpy one on an arbitrary x."""
    dims = (4, 4, 4, 4) if n == 2 else (4, 4, 2, 4)
    m0 = -0.2
    U = _links(dims, n, 93, oracle)
    b = oracle.restrict(_field(dims, n, 94), 0)
    x, info = oracle.cg_native(U, b, m0, tol=1e-11)
    _, info_py = oracle.cg(U, b, m0, tol=1e-11)
    assert info["iters"] == info_py["iters"]
    assert info["true_rel_residual"] <= 1e-11
    assert np.all(x[oracle.parity(dims) == 1] == 0)
    D = dense.dirac_matrix(U, m0)
    Dee, Deo, Doe, Doo = dense.schur_blocks(D, dims, n)
    S = Dee - Deo @ Doe / (4 + m0)
    e, _ = dense.parity_index(dims, n)
    xd = np.linalg.solve(S.conj().T @ S, b.ravel()[e])
    assert np.linalg.norm(x.ravel()[e] - xd) / np.linalg.norm(xd) < 1e-9
    y = _field(dims, n, 95)
    r_py = oracle.true_residual(U, b, y, m0)
    assert abs(oracle.true_residual_native(U, b, y, m0) - r_py) < 1e-13 * r_py
    # a dropped term in the operator would move the residual of the dense solution
    xs = np.zeros_like(b)
    xs.reshape(-1)[e] = xd
    assert oracle.true_residual_native(U, b, xs, m0) < 1e-11
