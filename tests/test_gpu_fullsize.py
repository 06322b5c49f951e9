"""Parity at the full sizes of the benchmarked configurations, in the launch
configuration the benchmark times:

* 48^4 SU(2) fundamental, heat-bath-like links (plaquette 0.6), m0 = -0.3:
  FP64 and FP32 hopping blocks, D^ and the plain D against the oracle on the
  whole lattice (norm-wise and largest per-site relative error);
  FP64 and mixed CG to 1e-10 checked by the oracle's FP64 residual.
* 32^4 adjoint (Haar links), m0 = -0.5: D^ and CG to 1e-10.
"""
import numpy as np
import pytest

from gpu_util import Field, requires_gpu, rel_err, site_rel_err, hrd

pytestmark = [pytest.mark.gpu, requires_gpu]


@pytest.fixture(scope="module")
def oracle():
    import oracle as O

    O._load()
    return O


@pytest.fixture(scope="module")
def f48():
    return Field((48, 48, 48, 48), "fund", seed=3, kind="smeared")


def test_48_hop_dhat_and_full(oracle, f48):
    h = hrd()
    dims, m0 = f48.dims, -0.3
    psi = f48.spinor(4)
    want = {"hop": oracle.hop_block(f48.U_orc, psi, 0), "dhat": oracle.dhat(f48.U_orc, oracle.restrict(psi, 0), m0),
            "full": oracle.dirac(f48.U_orc, psi, m0)}
    for prec, tol in (("f64", 1e-13), ("f32", 1e-6)):
        U = f48.U64 if prec == "f64" else f48.U32
        for kind, parity, sin, sout in (("hop", "hop_eo", "odd", "even"), ("dhat", "eo", "even", "even"),
                                        ("full", "full", "all", "all")):
            out = h.dirac_apply(U, f48.pack(psi, prec, sin), m0, "fund", parity, dims, prec=prec)
            got = f48.unpack(out, prec, sout)
            err, serr = rel_err(got, want[kind]), site_rel_err(got, want[kind])
            print(f"48^4 {kind} {prec}: rel_err {err:.3e} max_site_rel_err {serr:.3e}")
            assert err <= tol
            assert serr <= 10 * tol
            del out, got


def test_48_cg_both_modes(oracle, f48):
    h = hrd()
    dims, m0 = f48.dims, -0.3
    b = oracle.restrict(f48.spinor(4), 0)
    bp = f48.pack(b, "f64", "even")
    xs = {}
    U16 = h.convert_gauge_prec(f48.U64, dims, "fund", "f16")
    for mode in ("f64", "mixed", "mixed16"):
        x, info = h.cg_solve(f48.U64, bp, m0, 1e-10, dims, "fund", mode=mode,
                             U32=U16 if mode == "mixed16" else f48.U32)
        xe = f48.unpack(x, "f64", "even")
        res = oracle.true_residual_native(f48.U_orc, b, xe, m0)
        print(f"48^4 {mode}: {info} oracle residual {res:.3e}")
        assert res <= 1e-10
        xs[mode] = xe
    assert rel_err(xs["mixed"], xs["f64"]) < 1e-8
    assert rel_err(xs["mixed16"], xs["f64"]) < 1e-8


def test_32_adjoint_dhat_and_cg(oracle):
    h = hrd()
    dims, m0 = (32, 32, 32, 32), -0.5
    F = Field(dims, "adj", seed=2)
    b = oracle.restrict(F.spinor(22), 0)
    bp = F.pack(b, "f64", "even")
    out = h.dirac_apply(F.U64, bp, m0, "adj", "eo", dims)
    assert rel_err(F.unpack(out, "f64", "even"), oracle.dhat(F.U_orc, b, m0)) <= 1e-13
    for mode in ("f64", "mixed"):
        x, info = h.cg_solve(F.U64, bp, m0, 1e-10, dims, "adj", mode=mode, U32=F.U32)
        res = oracle.true_residual(F.U_orc, b, F.unpack(x, "f64", "even"), m0)
        print(f"32^4 adj {mode}: {info} oracle residual {res:.3e}")
        assert res <= 1e-10
