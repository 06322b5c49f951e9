"""GPU parity for SU(N > 2) with fermions in the fundamental, adjoint and
two-index representations (Sec. 1), through the dense link formats CPLX3,
CPLX4, CPLX6, CPLX10, REAL8 and REAL15 (SU(3): fundamental, adjoint,
symmetric, antisymmetric; SU(4): the same four).

* the library's representation of fundamental SU(3) / SU(4) links equals the
  oracle's map entry by entry (same bases) to FP64 rounding; pack/unpack of
  the dense formats round-trips exactly in FP64;
* D, D^ and the hop blocks with daggers equal the oracle on the oracle's own
  representation links: 1e-13 (FP64), 1e-6 (FP32), and for F16 the
  per-component / norm-wise bounds of the 16-bit format (oracle on the
  F16-rounded links and spinors);
* FP64, mixed and MIXED16 CG reach a true residual <= 1e-10 (oracle
  recomputation);
* the force d/dU Re<X, D[U] Y> and the action force with respect to the
  representation's links equal the oracle's to 1e-13 (real part for the
  real adjoint links); the chain rule of the representation map takes them
  to the fundamental links (oracle: automatic differentiation of its map).
"""
import numpy as np
import pytest
import torch

from gpu_util import FieldSUN, requires_gpu, rel_err, hrd, site_rel_err, to_dev_gauge
from paper_2411_18511_amd import inputs

pytestmark = [pytest.mark.gpu, requires_gpu]

CASES = [(3, "fund"), (3, "adj"), (3, "sym"), (3, "asym"), (4, "fund"), (4, "adj"), (4, "sym"), (4, "asym")]
LATS = [(4, 4, 4, 4), (6, 4, 6, 10), (2, 2, 2, 2), (4, 2, 2, 6)]


@pytest.fixture(scope="module")
def oracle():
    import oracle as O

    O._load()
    return O


@pytest.mark.parametrize("nc,rep", CASES)
def test_represent_and_pack(oracle, nc, rep):
    h = hrd()
    dims = (4, 2, 4, 6)
    F = FieldSUN(dims, nc, rep, seed=3)
    got = h.unpack_gauge(F.U64, dims, F.fmt, "f64").cpu().numpy()
    V = int(np.prod(dims))
    want = F.U_orc.reshape(4, V, F.n, F.n)
    if F.fmt in (h.REAL8, h.REAL15):
        want = want.real
    assert np.abs(got - want).max() < 1e-14
    # natural -> packed -> natural is exact in FP64
    nat = torch.from_numpy(np.ascontiguousarray(got)).cuda()
    again = h.unpack_gauge(h.pack_gauge(nat, dims, F.fmt, "f64"), dims, F.fmt, "f64").cpu().numpy()
    assert np.array_equal(again, got)
    # FP32 copy unpacks to the FP32 rounding
    g32 = h.unpack_gauge(F.U32, dims, F.fmt, "f32").cpu().numpy()
    if np.iscomplexobj(got):
        assert np.array_equal(g32.real, got.real.astype(np.float32).astype(np.float64))
        assert np.array_equal(g32.imag, got.imag.astype(np.float32).astype(np.float64))
    else:
        assert np.array_equal(g32, got.astype(np.float32).astype(np.float64))


def _round16_rep_links(F, oracle):
    """The library's F16 links as the oracle reads them: each entry of the
    library's FP64 representation links rounded through FP32 to binary16."""
    h = hrd()
    V = int(np.prod(F.dims))
    U = h.unpack_gauge(F.U64, F.dims, F.fmt, "f64").cpu().numpy().reshape((4,) + F.dims + (F.n, F.n))
    return oracle.round_links16(U).astype(np.complex128)


@pytest.mark.parametrize("nc,rep,dims", [(nc, r, d) for nc, r in CASES for d in LATS])
def test_operator_sun(oracle, nc, rep, dims):
    h = hrd()
    m0 = -0.3
    m = 4.0 + m0
    F = FieldSUN(dims, nc, rep, seed=11)
    U = F.U_orc
    psi = F.spinor(12)
    pe, po = oracle.restrict(psi, 0), oracle.restrict(psi, 1)
    for dagger in (False, True):
        want = {
            "full": (oracle.dirac_dagger if dagger else oracle.dirac)(U, psi, m0),
            "eo": (oracle.dhat_dagger if dagger else oracle.dhat)(U, pe, m0),
            "hop_eo": (oracle.hop_block_dagger if dagger else oracle.hop_block)(U, po, 0),
            "hop_oe": (oracle.hop_block_dagger if dagger else oracle.hop_block)(U, pe, 1),
        }
        src = {"full": (psi, "all"), "eo": (pe, "even"), "hop_eo": (po, "odd"), "hop_oe": (pe, "even")}
        osites = {"full": "all", "eo": "even", "hop_eo": "even", "hop_oe": "odd"}
        for prec, Ug, tol in (("f64", F.U64, 1e-13), ("f32", F.U32, 1e-6)):
            for par in ("full", "eo", "hop_eo", "hop_oe"):
                x, sites = src[par]
                out = h.dirac_apply(Ug, F.pack(x, prec, sites), m0, F.fmt, par, dims, prec=prec, dagger=dagger)
                w = want[par]
                if par == "hop_eo":
                    w = oracle.restrict(w, 0)
                if par == "hop_oe":
                    w = oracle.restrict(w, 1)
                err = rel_err(F.unpack(out, prec, osites[par]), w)
                assert err <= tol, (prec, par, dagger, err)
        # F16: oracle on the F16-rounded inputs, norm-wise bound of the 16-bit format
        Uq = _round16_rep_links(F, oracle)
        psiq = oracle.round_spinor16(psi)
        peq = oracle.restrict(psiq, 0)
        eps = 2.0 ** -12 * np.sqrt(8 * F.n)
        out = h.dirac_apply(F.U16, F.pack(psi, "f16", "all"), m0, F.fmt, "full", dims, prec="f16", dagger=dagger)
        w = (oracle.dirac_dagger if dagger else oracle.dirac)(Uq, psiq, m0)
        err = oracle.norm(F.unpack(out, "f16", "all") - w)
        assert err <= eps * oracle.norm(w) + 1e-5 * oracle.norm(w), ("f16 full", dagger)
        out = h.dirac_apply(F.U16, F.pack(pe, "f16", "even"), m0, F.fmt, "eo", dims, prec="f16", dagger=dagger)
        w = (oracle.dhat_dagger if dagger else oracle.dhat)(Uq, peq, m0)
        err = oracle.norm(F.unpack(out, "f16", "even") - w)
        bound = eps * (oracle.norm(w) + 16 * oracle.norm(peq) / m) + 1e-5 * oracle.norm(w)
        assert err <= bound, ("f16 eo", dagger, err, bound)


@pytest.mark.parametrize("nc,rep", CASES)
@pytest.mark.parametrize("mode", ["f64", "mixed", "mixed16"])
def test_cg_sun(oracle, nc, rep, mode):
    h = hrd()
    dims, m0 = (6, 4, 6, 10), -0.3
    F = FieldSUN(dims, nc, rep, seed=21, kind="smeared")
    b_np = oracle.restrict(F.spinor(22), 0)
    b = F.pack(b_np, "f64", "even")
    Ulo = {"f64": None, "mixed": F.U32, "mixed16": F.U16}[mode]
    x, info = h.cg_solve(F.U64, b, m0, 1e-10, dims, F.fmt, mode=mode, U32=Ulo)
    assert info["status"] == "HRD_OK" and info["true_rel_residual"] <= 1e-10
    xg = F.unpack(x, "f64", "even")
    assert oracle.true_residual(F.U_orc, b_np, xg, m0) <= 1e-10


def test_adjoint_su3_f64_many_blocks(oracle):
    """SU(3) adjoint (REAL8) FP64 operator on 16x8x8x16 (64 workgroups of the
    four-lanes-per-site kernel): hop blocks, D^ and their daggers against the
    oracle, and the FP64 CG (whose second D^+ stage fuses the residual update)
    to a true residual of 1e-10."""
    h = hrd()
    dims, m0 = (16, 8, 8, 16), -0.3
    F = FieldSUN(dims, 3, "adj", seed=31, kind="smeared")
    U = F.U_orc
    psi = F.spinor(32)
    pe, po = oracle.restrict(psi, 0), oracle.restrict(psi, 1)
    for dagger in (False, True):
        hb = oracle.hop_block_dagger if dagger else oracle.hop_block
        dh = oracle.dhat_dagger if dagger else oracle.dhat
        for par, x, sites, osites, want in (
                ("hop_eo", po, "odd", "even", oracle.restrict(hb(U, po, 0), 0)),
                ("hop_oe", pe, "even", "odd", oracle.restrict(hb(U, pe, 1), 1)),
                ("eo", pe, "even", "even", dh(U, pe, m0))):
            out = h.dirac_apply(F.U64, F.pack(x, "f64", sites), m0, F.fmt, par, dims, prec="f64", dagger=dagger)
            err = rel_err(F.unpack(out, "f64", osites), want)
            assert err <= 1e-13, (par, dagger, err)
    x, info = h.cg_solve(F.U64, F.pack(pe, "f64", "even"), m0, 1e-10, dims, F.fmt, mode="f64")
    assert info["status"] == "HRD_OK"
    assert oracle.true_residual(U, pe, F.unpack(x, "f64", "even"), m0) <= 1e-10


@pytest.mark.parametrize("rep", ["sym", "adj"])
def test_su4_f64_many_blocks(oracle, rep):
    """SU(4) symmetric (CPLX10) and adjoint (REAL15) FP64 operator on
    8x6x6x10 (1440 sites per parity: 22.5 workgroups of 64 sites of the
    four-lanes-per-site kernel, a ragged last one): hop blocks, D^ and their
    daggers against the oracle, and the FP64 CG (fused residual update and
    one norm partial per 64 sites) to a true residual of 1e-10."""
    h = hrd()
    dims, m0 = (8, 6, 6, 10), -0.3
    F = FieldSUN(dims, 4, rep, seed=33, kind="smeared")
    U = F.U_orc
    psi = F.spinor(34)
    pe, po = oracle.restrict(psi, 0), oracle.restrict(psi, 1)
    for dagger in (False, True):
        hb = oracle.hop_block_dagger if dagger else oracle.hop_block
        dh = oracle.dhat_dagger if dagger else oracle.dhat
        for par, x, sites, osites, want in (
                ("hop_eo", po, "odd", "even", oracle.restrict(hb(U, po, 0), 0)),
                ("hop_oe", pe, "even", "odd", oracle.restrict(hb(U, pe, 1), 1)),
                ("eo", pe, "even", "even", dh(U, pe, m0))):
            out = h.dirac_apply(F.U64, F.pack(x, "f64", sites), m0, F.fmt, par, dims, prec="f64", dagger=dagger)
            got = F.unpack(out, "f64", osites)
            err = rel_err(got, want)
            assert err <= 1e-13, (par, dagger, err)
            assert site_rel_err(got, want) <= 1e-12, (par, dagger)
    x, info = h.cg_solve(F.U64, F.pack(pe, "f64", "even"), m0, 1e-10, dims, F.fmt, mode="f64")
    assert info["status"] == "HRD_OK"
    assert oracle.true_residual(U, pe, F.unpack(x, "f64", "even"), m0) <= 1e-10


@pytest.mark.parametrize("nc,rep", CASES)
def test_force_sun(oracle, nc, rep):
    h = hrd()
    dims, m0 = (4, 2, 4, 6), -0.3
    F = FieldSUN(dims, nc, rep, seed=41)
    real = F.fmt in (h.REAL8, h.REAL15)
    V = int(np.prod(dims))

    def unpack_force(Fp):
        G = h.unpack_gauge(Fp, dims, F.fmt, "f64").cpu().numpy()
        return G.reshape((4,) + dims + (F.n, F.n))

    X, Y = F.spinor(42), F.spinor(43)
    got = unpack_force(h.dirac_force(F.U64, F.pack(X), F.pack(Y), dims, F.fmt, scale=0.7))
    want = 0.7 * oracle.force(X, Y, real_links=real)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    xi = oracle.restrict(F.spinor(44), 0)
    got = unpack_force(h.action_force(F.U64, F.pack(xi, "f64", "even"), m0, dims, F.fmt, scale=1.5))
    Xa, Ya = oracle.action_force_fields(F.U_orc, xi, m0)
    want = 1.5 * (2.0 / (4 + m0)) * oracle.force(Xa, Ya, real_links=real)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_sun_errors():
    h = hrd()
    dims = (4, 4, 4, 4)
    assert h.sun_rep_format(2, "sym") is None and h.sun_rep_format(5, "fund") is None
    assert h.sun_rep_format(4, "sym") == h.CPLX10 and h.sun_rep_format(4, "adj") == h.REAL15
    F = FieldSUN(dims, 3, "sym", seed=31)
    # the clover and batched paths take the SU(2) formats only
    with pytest.raises(h.HrdError) as e:
        h.clover_build(F.U64, 1.0, -0.2, dims, F.fmt)
    assert e.value.status == h.EINVAL


@pytest.mark.parametrize("dims", LATS)
def test_su3_two_row_format(oracle, dims):
    """SU(3) fundamental links stored as two rows: unpack reconstructs the third
    row, and the operator, CG and force equal those of the full links."""
    h = hrd()
    m0 = -0.3
    Uf = inputs.gauge_field_sun(dims, 51, 3)
    nat = to_dev_gauge(Uf)
    U64 = h.pack_gauge(nat, dims, "su3_row2", "f64")
    assert U64.numel() == int(np.prod(dims)) * 4 * 96
    back = h.unpack_gauge(U64, dims, "su3_row2", "f64").cpu().numpy().reshape(Uf.shape)
    assert np.abs(back - Uf).max() < 1e-14
    psi = inputs.gaussian_spinor(dims, 3, 52)
    pe = oracle.restrict(psi, 0)
    want = oracle.dhat(Uf, pe, m0)
    for prec, tol in (("f64", 1e-13), ("f32", 1e-6)):
        Ug = U64 if prec == "f64" else h.convert_gauge_prec(U64, dims, "su3_row2", prec)
        src = h.pack_spinor(torch.from_numpy(pe.reshape(-1, 4, 3)).cuda(), dims, "su3_row2", prec, "even")
        out = h.dirac_apply(Ug, src, m0, "su3_row2", "eo", dims, prec=prec)
        got = h.unpack_spinor(out, dims, "su3_row2", prec, "even").cpu().numpy().reshape(psi.shape)
        assert rel_err(got, want) <= tol, prec
        full = h.dirac_apply(Ug, h.pack_spinor(torch.from_numpy(psi.reshape(-1, 4, 3)).cuda(), dims, "su3_row2",
                                               prec, "all"), m0, "su3_row2", "full", dims, prec=prec, dagger=True)
        got = h.unpack_spinor(full, dims, "su3_row2", prec, "all").cpu().numpy().reshape(psi.shape)
        assert rel_err(got, oracle.dirac_dagger(Uf, psi, m0)) <= tol, prec
    b = h.pack_spinor(torch.from_numpy(pe.reshape(-1, 4, 3)).cuda(), dims, "su3_row2", "f64", "even")
    U16 = h.convert_gauge_prec(U64, dims, "su3_row2", "f16")
    x, info = h.cg_solve(U64, b, m0, 1e-10, dims, "su3_row2", mode="mixed16", U32=U16)
    xg = h.unpack_spinor(x, dims, "su3_row2", "f64", "even").cpu().numpy().reshape(psi.shape)
    assert info["true_rel_residual"] <= 1e-10 and oracle.true_residual(Uf, pe, xg, m0) <= 1e-10
    # the force is a general 3 x 3 matrix: written in the CPLX3 layout
    X, Y = inputs.gaussian_spinor(dims, 3, 53), inputs.gaussian_spinor(dims, 3, 54)
    Xp = h.pack_spinor(torch.from_numpy(X.reshape(-1, 4, 3)).cuda(), dims, "su3_row2", "f64", "all")
    Yp = h.pack_spinor(torch.from_numpy(Y.reshape(-1, 4, 3)).cuda(), dims, "su3_row2", "f64", "all")
    G = h.unpack_gauge(h.dirac_force(U64, Xp, Yp, dims, "su3_row2"), dims, "cplx3", "f64").cpu().numpy()
    wantG = oracle.force(X, Y)
    assert np.abs(G.reshape(wantG.shape) - wantG).max() <= 1e-13 * np.abs(wantG).max()


@pytest.mark.parametrize("nc,rep", CASES)
def test_represent_backward_sun(oracle, nc, rep):
    """Chain rule of the representation map on the GPU against the oracle's
    (automatic differentiation of its own map), for an arbitrary derivative
    G_rep, and the action force carried to the fundamental links: the GPU's
    dS/dR (action_force on the representation's links) through
    represent_backward_sun against the oracle's dS/dR through its chain rule."""
    h = hrd()
    dims, m0 = (4, 2, 4, 6), -0.3
    F = FieldSUN(dims, nc, rep, seed=61)
    real = F.fmt in (h.REAL8, h.REAL15)
    V = int(np.prod(dims))
    rng = np.random.default_rng(62)
    shape = (4,) + dims + (F.n, F.n)
    Gr = rng.standard_normal(shape) + (0 if real else 1j) * rng.standard_normal(shape)
    Uf64 = h.pack_gauge(to_dev_gauge(F.Uf), dims, "cplx3" if nc == 3 else "cplx4", "f64")
    nat = torch.from_numpy(np.ascontiguousarray(Gr.real if real else Gr).reshape(4, V, F.n, F.n)).cuda()
    Gf = h.represent_backward_sun(Uf64, h.pack_gauge(nat, dims, F.fmt, "f64"), dims, nc, rep)
    fund = "cplx3" if nc == 3 else "cplx4"
    got = h.unpack_gauge(Gf, dims, fund, "f64").cpu().numpy().reshape((4,) + dims + (nc, nc))
    want = oracle.represent_backward(F.Uf, Gr, rep)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    # dS/dU for S = phi^+ (D^+ D^)^-1 phi with the fermions in representation rep
    xi = oracle.restrict(F.spinor(63), 0)
    GR = h.action_force(F.U64, F.pack(xi, "f64", "even"), m0, dims, F.fmt)
    Gf = h.represent_backward_sun(Uf64, GR, dims, nc, rep)
    got = h.unpack_gauge(Gf, dims, fund, "f64").cpu().numpy().reshape((4,) + dims + (nc, nc))
    Xa, Ya = oracle.action_force_fields(F.U_orc, xi, m0)
    GR_orc = (2.0 / (4 + m0)) * oracle.force(Xa, Ya, real_links=real)
    want = oracle.represent_backward(F.Uf, GR_orc, rep)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_represent_backward_sun_errors():
    h = hrd()
    dims = (4, 4, 4, 4)
    F = FieldSUN(dims, 3, "adj", seed=64)
    Uf64 = h.pack_gauge(to_dev_gauge(F.Uf), dims, "cplx3", "f64")
    with pytest.raises(ValueError):
        h.represent_backward_sun(Uf64, F.U64, dims, 5, "sym")  # no SU(5) formats
    import ctypes

    st = h._lib.hrd_represent_backward_sun(ctypes.byref(h.lattice(dims)), 3, 1, Uf64.data_ptr(), F.U64.data_ptr(),
                                           Uf64.data_ptr(), None)
    assert st == h.EALIAS
