"""Links stored as the first row of the SU(2) matrix (HRD_FUND_SU2, and
HRD_ADJ_SU2 where the kernels compute the adjoint matrix from that row):
operator parity against the oracle (which uses the full fundamental matrices
and the trace formula of the adjoint map), solvers, force, batched launches,
and the packed layout."""
import numpy as np
import pytest
import torch

from gpu_util import tile_index, Field, from_dev_gauge, requires_gpu, rel_err, hrd

pytestmark = [pytest.mark.gpu, requires_gpu]

TOL = {"f64": 1e-13, "f32": 1e-6}


@pytest.fixture(scope="module")
def oracle():
    import oracle as O

    O._load()
    return O


_IN = {"full": "all", "eo": "even", "hop_eo": "odd", "hop_oe": "even"}
_OUT = {"full": "all", "eo": "even", "hop_eo": "even", "hop_oe": "odd"}


def _want(O, U, psi, m0, parity, dagger):
    if parity == "full":
        return O.dirac_dagger(U, psi, m0) if dagger else O.dirac(U, psi, m0)
    if parity == "eo":
        e = O.restrict(psi, 0)
        return O.dhat_dagger(U, e, m0) if dagger else O.dhat(U, e, m0)
    f = O.hop_block_dagger if dagger else O.hop_block
    return f(U, psi, 0 if parity == "hop_eo" else 1)


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 6, 10), (2, 2, 2, 2), (4, 24, 48, 48)])
@pytest.mark.parametrize("rep", ["fund_su2", "adj_su2"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("parity", ["full", "eo", "hop_eo", "hop_oe"])
@pytest.mark.parametrize("dagger", [False, True])
def test_su2_operator_parity(oracle, dims, rep, prec, parity, dagger):
    h = hrd()
    m0 = -0.3
    F = Field(dims, rep, seed=7, kind="smeared")
    psi = F.spinor(8)
    U = F.U64 if prec == "f64" else F.U32
    out = h.dirac_apply(U, F.pack(psi, prec, _IN[parity]), m0, rep, parity, dims, prec=prec, dagger=dagger)
    err = rel_err(F.unpack(out, prec, _OUT[parity]), _want(oracle, F.U_orc, psi, m0, parity, dagger))
    print(f"{dims} {rep} {prec} {parity} dag={dagger}: {err:.3e}")
    assert err <= TOL[prec]


def test_su2_layout_and_round_trip():
    h = hrd()
    dims = (6, 4, 6, 10)
    F = Field(dims, "fund_su2", seed=9)
    V = int(np.prod(dims))
    assert h.gauge_bytes(dims, "fund_su2", "f64") == V * 4 * 32
    assert h.gauge_bytes(dims, "adj_su2", "f32") == V * 4 * 16
    back = from_dev_gauge(h.unpack_gauge(F.U64, dims, "fund_su2", "f64"), dims)
    assert np.array_equal(back, F.Uf)  # exact: second row reconstructed from the first
    packed = F.U64.cpu().numpy().view(np.complex128)
    Vh = V // 2
    t, x1, x2, x3 = np.unravel_index(np.arange(V), dims)
    par = (t + x1 + x2 + x3) % 2
    idx = np.arange(V) >> 1
    for mu in range(4):
        flat = F.Uf[mu].reshape(V, 2, 2)
        for e in range(2):  # 64-site tiles of the two planes (U00, U01)
            assert np.array_equal(packed[(par * 4 + mu) * 2 * Vh + tile_index(Vh, idx, e, 2)], flat[:, 0, e])


@pytest.mark.parametrize("rep,m0", [("fund_su2", -0.3), ("adj_su2", -0.5)])
@pytest.mark.parametrize("mode", ["f64", "mixed"])
def test_su2_cg(oracle, rep, m0, mode):
    h = hrd()
    dims = (8, 8, 8, 8)
    F = Field(dims, rep, seed=11, kind="smeared")
    b = oracle.restrict(F.spinor(12), 0)
    x, info = h.cg_solve(F.U64, F.pack(b, "f64", "even"), m0, 1e-10, dims, rep, mode=mode, U32=F.U32)
    assert oracle.true_residual(F.U_orc, b, F.unpack(x, "f64", "even"), m0) <= 1e-10


@pytest.mark.parametrize("rep", ["fund_su2", "adj_su2"])
def test_su2_force_layout(oracle, rep):
    h = hrd()
    dims, m0 = (6, 4, 6, 10), -0.3
    F = Field(dims, rep, seed=13)
    xi = oracle.restrict(F.spinor(14), 0)
    G = h.action_force(F.U64, F.pack(xi, "f64", "even"), m0, dims, rep)
    base = "fund" if rep == "fund_su2" else "adj"
    got = from_dev_gauge(h.unpack_gauge(G, dims, base, "f64"), dims)
    X, Y = oracle.action_force_fields(F.U_orc, xi, m0)
    want = (2.0 / (4 + m0)) * oracle.force(X, Y, real_links=(base == "adj"))
    assert rel_err(got, want) <= 1e-13


def test_su2_batched_mixed_formats(oracle):
    h = hrd()
    specs = [((8, 8, 8, 8), "fund_su2", 3, -0.3), ((6, 4, 6, 10), "adj_su2", 2, -0.5), ((4, 4, 4, 4), "fund", 2, -0.2)]
    items = []
    for i, (dims, rep, nrhs, m0) in enumerate(specs):
        F = Field(dims, rep, seed=30 + i)
        psis = [oracle.restrict(F.spinor(40 + 10 * i + k), 0) for k in range(nrhs)]
        src = torch.stack([F.pack(q, "f32", "even") for q in psis])
        items.append((F, dims, rep, nrhs, m0, psis, src, torch.zeros_like(src)))
    probs = h.make_problems([{"dims": d, "rep": r, "nrhs": n, "m0": m, "U32": F.U32, "src": s, "dst": o}
                             for F, d, r, n, m, _, s, o in items])
    h.dirac_apply_batched(probs, "eo")
    torch.cuda.synchronize()
    for F, d, r, n, m, psis, s, o in items:
        for k in range(n):
            single = h.dirac_apply(F.U32, s[k], m, r, "eo", d, prec="f32")
            assert torch.equal(single, o[k])
        got = F.unpack(o[0], "f32", "even")
        assert rel_err(got, oracle.dhat(F.U_orc, psis[0], m)) <= 1e-6
