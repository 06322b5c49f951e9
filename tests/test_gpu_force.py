"""GPU parity of the fermion force (derivative of Re<X, D[U] Y> with respect to
the links; the HMC force of the paper's Sec. 2.1 setting) and of the chain rule
through the adjoint map, against the oracle: 1e-13 on identical inputs."""
import numpy as np
import pytest

from gpu_util import Field, from_dev_gauge, requires_gpu, hrd

pytestmark = [pytest.mark.gpu, requires_gpu]


@pytest.fixture(scope="module")
def oracle():
    import oracle as O

    O._load()
    return O


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 6, 10), (2, 2, 2, 2)])
@pytest.mark.parametrize("rep", ["fund", "adj"])
def test_force_parity(oracle, dims, rep):
    h = hrd()
    F = Field(dims, rep, seed=61)
    X, Y = F.spinor(62), F.spinor(63)
    G = h.dirac_force(F.U64, F.pack(X), F.pack(Y), dims, rep, scale=0.7)
    got = from_dev_gauge(h.unpack_gauge(G, dims, rep, "f64"), dims)
    want = 0.7 * oracle.force(X, Y, real_links=(rep == "adj"))
    err = _rel(got, want)
    print(f"force {dims} {rep} rel_err={err:.3e}")
    assert err <= 1e-13


@pytest.mark.parametrize("dims,rep,m0", [((8, 8, 8, 8), "fund", -0.2), ((6, 4, 6, 10), "adj", -0.4)])
def test_action_force_parity(oracle, dims, rep, m0):
    """Same xi on both sides: the assembly (2/m) G[X, Y] with the X, Y built from xi."""
    h = hrd()
    F = Field(dims, rep, seed=71)
    xi = oracle.restrict(F.spinor(72), 0)
    G = h.action_force(F.U64, F.pack(xi, "f64", "even"), m0, dims, rep, scale=1.5)
    got = from_dev_gauge(h.unpack_gauge(G, dims, rep, "f64"), dims)
    X, Y = oracle.action_force_fields(F.U_orc, xi, m0)
    want = 1.5 * (2.0 / (4 + m0)) * oracle.force(X, Y, real_links=(rep == "adj"))
    assert _rel(got, want) <= 1e-13


@pytest.mark.parametrize("dims", [(6, 4, 6, 10)])
def test_represent_backward(oracle, dims):
    """dL/dU for L = sum g_ab R_ab(U) against the directional derivative of R."""
    h = hrd()
    F = Field(dims, "adj", seed=81)
    rng = np.random.default_rng(82)
    g = rng.standard_normal((4,) + dims + (3, 3))
    from gpu_util import to_dev_gauge

    g_dev = h.pack_gauge(to_dev_gauge(g), dims, "adj", "f64")
    Gf = from_dev_gauge(h.unpack_gauge(h.represent_backward(F.Uf64, g_dev, dims), dims, "fund", "f64"), dims)
    # exact first-order check with the oracle's adjoint map: R is quadratic in U,
    # so a central difference is exact up to rounding
    E = rng.standard_normal(F.Uf.shape) + 1j * rng.standard_normal(F.Uf.shape)
    eps = 1e-3
    Rp = oracle.represent_adjoint(F.Uf + eps * E)
    Rm = oracle.represent_adjoint(F.Uf - eps * E)
    fd = np.sum(g * (Rp - Rm)) / (2 * eps)
    an = np.real(np.sum(np.conj(Gf) * E))
    assert abs(fd - an) <= 1e-10 * abs(an)
