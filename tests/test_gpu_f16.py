"""GPU parity of the 16-bit storage path (binary16 spinors with a per-site FP32
scale, binary16 links, FP32 arithmetic) and of the CG whose inner iterations
use it.

* the encoder is bit-exact against the oracle's definition of the format
  (spinors: codes and scales; links: every entry), both sides taking the
  rounding decisions in FP32;
* the operator in F16 equals the FP64 oracle applied to the F16-rounded
  inputs, within the bound of the output re-encoding: per real component
  |got - want| <= s 2^-12 + 1e-5 s_want for a single hop (s the output site
  scale), and, for D^ with its re-encoded intermediate t, norm-wise
  eps (||want|| + 16 ||psi|| / m) + 1e-5 ||want||, eps = 2^-12 sqrt(8N)
  (the worst-case binary16 rounding of a site, ||D_eo||, ||D_oe|| <= 4);
* the MIXED16 CG reaches a true residual <= 1e-10 (oracle recomputation),
  also with the clover term.
"""
import numpy as np
import pytest
import torch

from gpu_util import Field, requires_gpu, rel_err, hrd, to_dev_spinor

pytestmark = [pytest.mark.gpu, requires_gpu]

REPS = ["fund", "adj", "fund_su2", "adj_su2"]


@pytest.fixture(scope="module")
def oracle():
    import oracle as O

    O._load()
    return O


def parity_sites(dims, p, oracle):
    par = oracle.parity(dims).reshape(-1)
    return np.nonzero(par == p)[0]  # lex order == eo index order


def decode_spinor16(raw, dims, n, nparity):
    """Host decoder of the documented F16 spinor layout (64-site tiles of N
    planes followed by the tile's FP32 site scales): returns (codes
    [nparity, Vh, 4, n, 2] float16, scales [nparity, Vh] float32)."""
    Vh = int(np.prod(dims)) // 2
    nc = 4 * n
    P = nc // 4
    blk = Vh * (4 * nc + 4)
    b = raw.cpu().numpy().view(np.uint8)
    site = np.arange(Vh)
    b0 = site & ~63
    nb = np.minimum(64, Vh - b0)
    tile = b0 * (16 * P + 4)  # byte offset of each site's 64-site tile
    codes, scales = [], []
    for q in range(nparity):
        part = b[q * blk:(q + 1) * blk]
        planes = np.stack([part[(tile + (k * nb + site - b0) * 16)[:, None] + np.arange(16)] for k in range(P)])
        c = planes.view(np.float16).reshape(P, Vh, 8).transpose(1, 0, 2).reshape(Vh, nc, 2).reshape(Vh, 4, n, 2)
        codes.append(c)
        sc = part[(tile + P * nb * 16 + (site - b0) * 4)[:, None] + np.arange(4)]
        scales.append(sc.view(np.float32).reshape(Vh))
    return np.stack(codes), np.stack(scales)


@pytest.mark.parametrize("n,dims", [(2, (4, 4, 4, 4)), (3, (6, 4, 6, 10)), (2, (4, 24, 48, 48))])
def test_spinor_encoder_bit_exact(oracle, n, dims):
    h = hrd()
    rep = "fund" if n == 2 else "adj"
    F = Field(dims, rep, seed=5)
    psi = F.spinor(6)
    psi[1, 1, 1, 1] = 0  # a zero site
    psi[0, 0, 0, 0] *= 1e-30  # a tiny site (scale far below 1)
    p64 = F.pack(psi, "f64", "all")
    p16 = h.convert_spinor_prec(p64, dims, rep, 2, "f64", "f16")
    codes, scales = decode_spinor16(p16, dims, n, 2)
    flat = psi.reshape(-1, 4, n)
    for p in (0, 1):
        want_c, want_s = oracle.quantize_spinor16(flat[parity_sites(dims, p, oracle)])
        assert np.array_equal(scales[p], want_s)
        assert np.array_equal(codes[p].view(np.uint16), want_c.view(np.uint16))
    # F16 -> F64 gives exactly the represented values; F16 -> F32 -> F64 rounds once
    back = F.unpack(h.convert_spinor_prec(p16, dims, rep, 2, "f16", "f64"), "f64", "all")
    assert np.array_equal(back, oracle.round_spinor16(psi))
    b32 = F.unpack(h.convert_spinor_prec(h.convert_spinor_prec(p16, dims, rep, 2, "f16", "f32"), dims, rep, 2,
                                         "f32", "f64"), "f64", "all")
    assert rel_err(b32, back) < 1e-7


def decode_links16(raw, dims, rep):
    """Host decoder of the documented F16 gauge layouts -> float64 entries per (p, mu, site)."""
    Vh = int(np.prod(dims)) // 2
    b = raw.cpu().numpy().view(np.uint8)
    out = []
    for pm in range(8):
        if rep in ("fund_su2", "adj_su2"):
            blk = b[pm * Vh * 8:(pm + 1) * Vh * 8].view(np.float16).reshape(Vh, 4)
            out.append(blk.astype(np.float64))
        elif rep == "fund":
            blk = b[pm * Vh * 16:(pm + 1) * Vh * 16].view(np.float16).reshape(Vh, 8)
            out.append(blk.astype(np.float64))
        else:  # 64-site tiles: the tile's 16-byte planes, then its entries 8
            blk = b[pm * Vh * 18:(pm + 1) * Vh * 18]
            site = np.arange(Vh)
            b0 = site & ~63
            nb = np.minimum(64, Vh - b0)
            tile = b0 * 18
            e = blk[(tile + (site - b0) * 16)[:, None] + np.arange(16)].view(np.float16).reshape(Vh, 8)
            e8 = blk[(tile + nb * 16 + (site - b0) * 2)[:, None] + np.arange(2)].view(np.float16).reshape(Vh, 1)
            out.append(np.concatenate([e, e8], axis=1).astype(np.float64))
    return out


@pytest.mark.parametrize("rep", REPS)
def test_link_encoder_bit_exact(oracle, rep):
    h = hrd()
    dims = (4, 4, 6, 2)
    F = Field(dims, rep, seed=7)
    U16 = h.convert_gauge_prec(F.U64, dims, rep, "f16")
    got = decode_links16(U16, dims, rep)
    if rep in ("fund_su2", "adj_su2", "fund"):
        ref = oracle.round_links16(F.Uf)
    else:
        ref = oracle.round_links16(oracle.represent_adjoint(F.Uf))
    V = int(np.prod(dims))
    for p in (0, 1):
        sites = parity_sites(dims, p, oracle)
        for mu in range(4):
            R = ref[mu].reshape(V, *ref.shape[-2:])[sites]
            if rep in ("fund_su2", "adj_su2"):
                want = np.stack([R[:, 0, 0].real, R[:, 0, 0].imag, R[:, 0, 1].real, R[:, 0, 1].imag], axis=1)
            elif rep == "fund":
                want = np.stack([f(R[:, i, j]) for i in range(2) for j in range(2) for f in (np.real, np.imag)],
                                axis=1)
            else:
                want = R.reshape(len(sites), 9)
            g = got[4 * p + mu]
            if rep == "adj":
                # the adjoint links are formed on the GPU in FP64 first: the FP32 rounding may
                # differ in the last bit, so allow one binary16 step on rare entries
                d = np.abs(g - want)
                assert d.max() <= 2.0 ** -10 and np.mean(d > 0) < 1e-3
            else:
                assert np.array_equal(g, want)


def _oracle_inputs(F, oracle, psi):
    """F16-rounded oracle inputs: the spinor as stored, the links of the operator as stored."""
    if F.rep == "adj":
        U = oracle.round_links16(oracle.represent_adjoint(F.Uf)).astype(np.complex128)
    elif F.rep == "adj_su2":
        U = oracle.represent_adjoint(oracle.round_links16(F.Uf)).astype(np.complex128)
    else:
        U = oracle.round_links16(F.Uf)
    return U, oracle.round_spinor16(psi)


def _site_bound_check(got, want, n):
    """Per real component: |got - want| <= s 2^-12 + 1e-5 s_want, s = site scale of got (binary16
    re-encoding of the output, plus the FP32 arithmetic of the kernel)."""
    g = got.reshape(-1, 4 * n)
    w = want.reshape(-1, 4 * n)
    s = np.maximum(np.abs(g.real), np.abs(g.imag)).max(axis=1, keepdims=True)
    sw = np.maximum(np.abs(w.real), np.abs(w.imag)).max(axis=1, keepdims=True)
    bound = s * 2.0 ** -12 + 1e-5 * sw + 1e-300
    err = np.maximum(np.abs(g.real - w.real), np.abs(g.imag - w.imag))
    return float((err / bound).max())


@pytest.mark.parametrize("rep,dims", [(r, d) for r in REPS for d in [(4, 4, 4, 4), (6, 4, 6, 10), (4, 24, 48, 48), (2, 2, 2, 2), (4, 2, 2, 6)]])
def test_operator_f16(oracle, rep, dims):
    h = hrd()
    m0 = -0.3
    m = 4.0 + m0
    F = Field(dims, rep, seed=11, kind="smeared")
    n = F.n
    U16 = h.convert_gauge_prec(F.U64, dims, rep, "f16")
    psi = F.spinor(12)
    Uq, psiq = _oracle_inputs(F, oracle, psi)
    p16_all = h.convert_spinor_prec(F.pack(psi, "f64", "all"), dims, rep, 2, "f64", "f16")
    pe = oracle.restrict(psi, 0)
    po = oracle.restrict(psi, 1)
    pe16 = h.convert_spinor_prec(F.pack(pe, "f64", "even"), dims, rep, 1, "f64", "f16")
    po16 = h.convert_spinor_prec(F.pack(po, "f64", "odd"), dims, rep, 1, "f64", "f16")
    peq, poq = oracle.restrict(psiq, 0), oracle.restrict(psiq, 1)

    def back(t, sites, nparity):
        return F.unpack(h.convert_spinor_prec(t, dims, rep, nparity, "f16", "f64"), "f64", sites)

    for dagger in (False, True):
        # single hops: per-component bound
        out = h.dirac_apply(U16, po16, m0, rep, "hop_eo", dims, prec="f16", dagger=dagger)
        f = oracle.hop_block_dagger if dagger else oracle.hop_block
        want = oracle.restrict(f(Uq, poq, 0), 0)
        got = back(out, "even", 1)
        par = oracle.parity(dims) == 0
        assert _site_bound_check(got[par], want[par], n) <= 1.0, ("hop_eo", dagger)
        out = h.dirac_apply(U16, pe16, m0, rep, "hop_oe", dims, prec="f16", dagger=dagger)
        want = oracle.restrict(f(Uq, peq, 1), 1)
        got = back(out, "odd", 1)
        assert _site_bound_check(got[~par], want[~par], n) <= 1.0, ("hop_oe", dagger)
        # full D: one launch, per-component bound
        out = h.dirac_apply(U16, p16_all, m0, rep, "full", dims, prec="f16", dagger=dagger)
        want = (oracle.dirac_dagger if dagger else oracle.dirac)(Uq, psiq, m0)
        assert _site_bound_check(back(out, "all", 2), want, n) <= 1.0, ("full", dagger)
        # D^: re-encoded intermediate, norm-wise bound
        out = h.dirac_apply(U16, pe16, m0, rep, "eo", dims, prec="f16", dagger=dagger)
        want = (oracle.dhat_dagger if dagger else oracle.dhat)(Uq, peq, m0)
        got = back(out, "even", 1)
        eps = 2.0 ** -12 * np.sqrt(8 * n)
        bound = eps * (oracle.norm(want) + 16 * oracle.norm(peq) / m) + 1e-5 * oracle.norm(want)
        err = oracle.norm(got - want)
        assert err <= bound, ("eo", dagger, err, bound)
        # and in practice far inside it
        assert err <= 0.25 * bound


@pytest.mark.parametrize("rep", REPS)
def test_cg_mixed16(oracle, rep):
    h = hrd()
    dims, m0 = (6, 4, 6, 10), -0.3
    F = Field(dims, rep, seed=21, kind="smeared")
    U16 = h.convert_gauge_prec(F.U64, dims, rep, "f16")
    b_np = oracle.restrict(F.spinor(22), 0)
    b = F.pack(b_np, "f64", "even")
    x, info = h.cg_solve(F.U64, b, m0, 1e-10, dims, rep, mode="mixed16", U32=U16)
    assert info["status"] == "HRD_OK" and info["true_rel_residual"] <= 1e-10
    assert info["reliable_updates"] >= 1
    xg = F.unpack(x, "f64", "even")
    assert oracle.true_residual(F.U_orc, b_np, xg, m0) <= 1e-10
    xo, _ = oracle.cg(F.U_orc, b_np, m0, tol=1e-12)
    assert rel_err(xg, xo) < 1e-7


def test_cg_mixed16_large(oracle):
    h = hrd()
    dims, m0 = (4, 24, 48, 48), -0.3
    F = Field(dims, "fund_su2", seed=31, kind="smeared")
    U16 = h.convert_gauge_prec(F.U64, dims, "fund_su2", "f16")
    b_np = oracle.restrict(F.spinor(32), 0)
    b = F.pack(b_np, "f64", "even")
    x, info = h.cg_solve(F.U64, b, m0, 1e-10, dims, "fund_su2", mode="mixed16", U32=U16)
    assert info["true_rel_residual"] <= 1e-10
    assert oracle.true_residual(F.U_orc, b_np, F.unpack(x, "f64", "even"), m0) <= 1e-10
    x32, i32 = h.cg_solve(F.U64, b, m0, 1e-10, dims, "fund_su2", mode="mixed", U32=F.U32)
    assert rel_err(F.unpack(x, "f64", "even"), F.unpack(x32, "f64", "even")) < 1e-7
    print("iters mixed16", info["iters"], info["reliable_updates"], "mixed", i32["iters"], i32["reliable_updates"])


@pytest.mark.parametrize("kind", ["sw", "exp"])
def test_clover_cg_mixed16(oracle, kind):
    h = hrd()
    dims, m0, csw = (6, 4, 6, 10), -0.3, 1.4
    F = Field(dims, "fund", seed=41, kind="smeared")
    c64 = h.clover_build(F.U64, csw, m0, dims, "fund", kind=kind)
    c32 = h.convert_clover(c64, dims, "fund")
    U16 = h.convert_gauge_prec(F.U64, dims, "fund", "f16")
    b_np = oracle.restrict(F.spinor(42), 0)
    b = F.pack(b_np, "f64", "even")
    x, info = h.cg_solve_clover(F.U64, c64, b, 1e-10, dims, "fund", mode="mixed16", U32=U16, clov32=c32)
    assert info["true_rel_residual"] <= 1e-10
    assert oracle.true_residual_clover(F.U_orc, b_np, F.unpack(x, "f64", "even"), m0, csw, kind) <= 1e-10


def test_f16_errors():
    h = hrd()
    dims = (4, 4, 4, 4)
    F = Field(dims, "fund", seed=51)
    with pytest.raises(h.HrdError) as e:
        h.convert_gauge_prec(F.U64, dims, "fund", "f64")
    assert e.value.status == h.EINVAL
    psi = F.pack(F.spinor(52), "f64", "even")
    p16 = h.convert_spinor_prec(psi, dims, "fund", 1, "f64", "f16")
    # level-1 BLAS does not take F16 fields
    with pytest.raises(h.HrdError) as e:
        h.blas_norm2(p16, dims, "fund", "f16", 1)
    assert e.value.status == h.EINVAL
    # mixed16 without the F16 gauge field
    with pytest.raises(h.HrdError) as e:
        h.cg_solve(F.U64, psi, -0.2, 1e-10, dims, "fund", mode="mixed16")
    assert e.value.status == h.EINVAL
