"""GPU parity of the Wilson-Dirac operator (Sec. 2.1 of the paper: the plain
unimproved operator and its even/odd preconditioned form) against the oracle,
through the C ABI.

Tolerances (norm-wise relative, ||y_gpu - y_orc|| / ||y_orc||): 1e-13 in FP64,
1e-6 in FP32 where the oracle runs on the original FP64 inputs (FP32 input
rounding ~6e-8 per entry plus ~8-term sums).  The largest per-site relative
error is reported beside it and bounded by 10x the norm-wise tolerance (a
site's norm is rarely below a third of the field's root mean square for
Gaussian spinors of 16 or more real components).  Lattices span several 256-site
tiles with ragged tails and asymmetric extents; 2^4 is the degenerate case
where forward and backward neighbours coincide; 4x24x48x48 is swept in x1-slabs
narrower than L1 (the traversal used at 48^4).
"""
import numpy as np
import pytest

from gpu_util import tile_index, Field, from_dev_gauge, requires_gpu, rel_err, site_rel_err, hrd

pytestmark = [pytest.mark.gpu, requires_gpu]

TOL = {"f64": 1e-13, "f32": 1e-6}
LATTICES = [(8, 8, 8, 8), (6, 4, 6, 10), (2, 2, 2, 2), (4, 2, 2, 6), (4, 24, 48, 48)]


@pytest.fixture(scope="module")
def oracle():
    import oracle as O

    O._load()
    return O


def _oracle_apply(O, U, psi, m0, parity, dagger):
    if parity == "full":
        return O.dirac_dagger(U, psi, m0) if dagger else O.dirac(U, psi, m0)
    if parity == "eo":
        e = O.restrict(psi, 0)
        return O.dhat_dagger(U, e, m0) if dagger else O.dhat(U, e, m0)
    if parity == "hop_eo":  # out_e = D_eo psi_o ; dagger: g5 D_eo g5
        f = O.hop_block_dagger if dagger else O.hop_block
        return f(U, psi, 0)
    f = O.hop_block_dagger if dagger else O.hop_block
    return f(U, psi, 1)


_IN_SITES = {"full": "all", "eo": "even", "hop_eo": "odd", "hop_oe": "even"}
_OUT_SITES = {"full": "all", "eo": "even", "hop_eo": "even", "hop_oe": "odd"}


@pytest.mark.parametrize("dims", LATTICES)
@pytest.mark.parametrize("rep", ["fund", "adj"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("parity", ["full", "eo", "hop_eo", "hop_oe"])
@pytest.mark.parametrize("dagger", [False, True])
def test_dirac_apply_parity(oracle, dims, rep, prec, parity, dagger):
    h = hrd()
    m0 = -0.2 if rep == "fund" else -0.5
    F = Field(dims, rep, seed=1)
    psi = F.spinor(2)
    U = F.U64 if prec == "f64" else F.U32
    src = F.pack(psi, prec, _IN_SITES[parity])
    out = h.dirac_apply(U, src, m0, rep, parity, dims, prec=prec, dagger=dagger)
    got = F.unpack(out, prec, _OUT_SITES[parity])
    want = _oracle_apply(oracle, F.U_orc, psi, m0, parity, dagger)
    err = rel_err(got, want)
    serr = site_rel_err(got, want)
    print(f"dims={dims} rep={rep} prec={prec} parity={parity} dagger={dagger} rel_err={err:.3e} "
          f"max_site_rel_err={serr:.3e}")
    assert err <= TOL[prec]
    assert serr <= 10 * TOL[prec]


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 6, 10)])
@pytest.mark.parametrize("rep", ["fund", "adj"])
def test_pack_round_trip_and_layout(dims, rep):
    h = hrd()
    F = Field(dims, rep, seed=3)
    psi = F.spinor(4)
    for sites in ("all", "even", "odd"):
        packed = F.pack(psi, "f64", sites)
        back = F.unpack(packed, "f64", sites)
        import oracle as O

        if sites == "all":
            assert np.array_equal(back, psi)
        else:
            par = 0 if sites == "even" else 1
            assert np.array_equal(back, O.restrict(psi, par))
    # documented layout: F64 full field [parity][64-site tiles of component
    # planes], site index lex >> 1
    packed = F.pack(psi, "f64", "all").cpu().numpy().view(np.complex128)
    V = int(np.prod(dims))
    Vh = V // 2
    NC = 4 * F.n
    flat = psi.reshape(V, NC)
    t, x1, x2, x3 = np.unravel_index(np.arange(V), dims)
    par = (t + x1 + x2 + x3) % 2
    idx = np.arange(V) >> 1
    for k in range(NC):
        assert np.array_equal(packed[par * NC * Vh + tile_index(Vh, idx, k, NC)], flat[:, k])
    # F32: planes of component pairs, same tiles
    p32 = F.pack(psi, "f32", "all").cpu().numpy().view(np.complex64)
    for k in range(NC):
        pos = (par * (NC // 2) * Vh + tile_index(Vh, idx, k // 2, NC // 2)) * 2 + (k % 2)
        assert np.array_equal(p32[pos], flat[:, k].astype(np.complex64))
    # gauge round trip
    if rep == "fund":
        back = from_dev_gauge(h.unpack_gauge(F.U64, dims, "fund", "f64"), dims)
        assert np.array_equal(back, F.Uf)
    else:
        back = from_dev_gauge(h.unpack_gauge(F.U64, dims, "adj", "f64"), dims)
        assert np.abs(back - F.U_orc.real).max() < 1e-15


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 6, 10)])
def test_represent_parity(oracle, dims):
    h = hrd()
    F = Field(dims, "adj", seed=5)
    R = from_dev_gauge(h.unpack_gauge(F.U64, dims, "adj", "f64"), dims)
    want = oracle.represent_adjoint(F.Uf)
    assert np.abs(R - want).max() < 1e-15
    R32 = from_dev_gauge(h.unpack_gauge(F.U32, dims, "adj", "f32"), dims)
    assert np.abs(R32 - want).max() < 1e-7


def test_convert_spinor_round_trip():
    h = hrd()
    dims = (6, 4, 6, 10)
    F = Field(dims, "fund", seed=6)
    psi = F.spinor(7)
    p64 = F.pack(psi, "f64", "all")
    p32 = h.convert_spinor(p64, dims, "fund", 2, True)
    direct32 = F.pack(psi, "f32", "all")
    assert np.array_equal(p32.cpu().numpy(), direct32.cpu().numpy())
    back = h.convert_spinor(p32, dims, "fund", 2, False)
    got = F.unpack(back, "f64", "all")
    assert np.array_equal(got, psi.astype(np.complex64).astype(np.complex128))
