"""Autograd wrappers of the library (the HMC force of the paper's Sec. 2.1
setting): gradients against the oracle's force and D^+, and the fermion-action
gradient against central finite differences (eps = 1e-6) of the action
computed with dense solves at 4^4, for fundamental and adjoint fermions."""
import numpy as np
import pytest
import torch

from gpu_util import Field, from_dev_gauge, from_dev_spinor, requires_gpu, to_dev_gauge, to_dev_spinor, hrd
from paper_2411_18511_amd import inputs

pytestmark = [pytest.mark.gpu, requires_gpu]


@pytest.fixture(scope="module")
def oracle():
    import oracle as O

    O._load()
    return O


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("rep", ["fund", "adj"])
def test_dirac_apply_backward(oracle, rep):
    from paper_2411_18511_amd import autograd as AG

    dims, m0 = (6, 4, 6, 10), -0.3
    F = Field(dims, rep, seed=91)
    U_nat = to_dev_gauge(F.Uf if rep == "fund" else F.U_orc.real)
    U_nat.requires_grad_(True)
    psi = F.spinor(92)
    psi_t = to_dev_spinor(psi).requires_grad_(True)
    y = AG.dirac_apply(U_nat, psi_t, dims, rep, m0)
    assert _rel(from_dev_spinor(y.detach(), dims), oracle.dirac(F.U_orc, psi, m0)) < 1e-13
    g = F.spinor(93)
    y.backward(to_dev_spinor(g))
    want_psi = oracle.dirac_dagger(F.U_orc, g, m0)
    assert _rel(from_dev_spinor(psi_t.grad, dims), want_psi) < 1e-13
    want_U = oracle.force(g, psi, real_links=(rep == "adj"))
    assert _rel(from_dev_gauge(U_nat.grad, dims), want_U) < 1e-13


def _dense_action(oracle, Uf, phi_vec, m0, dims, n):
    from oracle import dense

    U = Uf if n == 2 else oracle.represent_adjoint(Uf).astype(np.complex128)
    D = dense.dirac_matrix(U, m0)
    Dee, Deo, Doe, Doo = dense.schur_blocks(D, dims, n)
    Dh = Dee - Deo @ Doe / (4 + m0)
    y = np.linalg.solve(Dh.conj().T, phi_vec)
    return float(np.real(np.vdot(y, y)))


@pytest.mark.parametrize("rep", ["fund", "adj"])
@pytest.mark.parametrize("mode", ["f64", "mixed"])
def test_fermion_action_central_differences(oracle, rep, mode):
    from oracle import dense
    from paper_2411_18511_amd import autograd as AG

    dims, m0 = (4, 4, 4, 4), -0.4
    n = 2 if rep == "fund" else 3
    Uf = inputs.gauge_field(dims, 95)
    phi = oracle.restrict(inputs.gaussian_spinor(dims, n, 96), 0)
    U_t = to_dev_gauge(Uf).requires_grad_(True)
    phi_t = to_dev_spinor(phi)
    S = AG.fermion_action(U_t, phi_t, dims, rep, m0, 1e-12, mode)
    S.backward()
    grad = from_dev_gauge(U_t.grad, dims)
    e, _ = dense.parity_index(dims, n)
    phi_vec = phi.ravel()[e]
    S_dense = _dense_action(oracle, Uf, phi_vec, m0, dims, n)
    assert abs(float(S) - S_dense) < 1e-10 * abs(S_dense)
    rng = np.random.default_rng(97)
    eps = 1e-6
    for _ in range(6):
        E = rng.standard_normal(Uf.shape) + 1j * rng.standard_normal(Uf.shape)
        fd = (_dense_action(oracle, Uf + eps * E, phi_vec, m0, dims, n)
              - _dense_action(oracle, Uf - eps * E, phi_vec, m0, dims, n)) / (2 * eps)
        an = float(np.real(np.sum(np.conj(grad) * E)))
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-7, (fd, an)


def test_fermion_action_phi_gradient(oracle):
    from paper_2411_18511_amd import autograd as AG

    dims, m0 = (4, 4, 4, 4), -0.2
    Uf = inputs.gauge_field(dims, 98)
    phi = oracle.restrict(inputs.gaussian_spinor(dims, 2, 99), 0)
    phi_t = to_dev_spinor(phi).requires_grad_(True)
    S = AG.fermion_action(to_dev_gauge(Uf), phi_t, dims, "fund", m0, 1e-12)
    S.backward()
    xi, _ = oracle.cg(Uf, phi, m0, tol=1e-12)
    assert _rel(from_dev_spinor(phi_t.grad, dims), 2 * xi) < 1e-9


def test_config5_force_assembly_full_size(oracle):
    """24^3 x 48 adjoint, m0 = -0.4: the GPU solve reaches residual 1e-10 (oracle
    recomputation) and the GPU action force equals the oracle's force built
    from that same solution."""
    dims, m0 = (48, 24, 24, 24), -0.4
    F = Field(dims, "adj", seed=5)
    phi = oracle.restrict(F.spinor(55), 0)
    b = F.pack(phi, "f64", "even")
    x, info = hrd().cg_solve(F.U64, b, m0, 1e-10, dims, "adj", mode="mixed", U32=F.U32)
    xi = F.unpack(x, "f64", "even")
    assert oracle.true_residual(F.U_orc, phi, xi, m0) <= 1e-10
    G = hrd().action_force(F.U64, x, m0, dims, "adj")
    got = from_dev_gauge(hrd().unpack_gauge(G, dims, "adj", "f64"), dims)
    X, Y = oracle.action_force_fields(F.U_orc, xi, m0)
    want = (2.0 / (4 + m0)) * oracle.force(X, Y, real_links=True)
    assert _rel(got, want) <= 1e-13
