"""Parity at the full sizes of the benchmarked configurations, in the launch
configuration the benchmark times:

* 48^4 SU(2) fundamental, heat-bath-like links (plaquette 0.6), m0 = -0.3:
  FP64 and FP32 hopping blocks and D^ against the oracle on the whole lattice;
  FP64 and mixed CG to 1e-10 checked by the oracle's FP64 residual.
* 32^4 adjoint (Haar links), m0 = -0.5: D^ and CG to 1e-10.
"""
import numpy as np
import pytest

from gpu_util import Field, requires_gpu, rel_err, hrd

pytestmark = [pytest.mark.gpu, requires_gpu]


@pytest.fixture(scope="module")
def oracle():
    import oracle as O

    O._load()
    return O


@pytest.fixture(scope="module")
def f48():
    return Field((48, 48, 48, 48), "fund", seed=3, kind="smeared")


def test_48_hop_and_dhat(oracle, f48):
    h = hrd()
    dims, m0 = f48.dims, -0.3
    psi = f48.spinor(4)
    for prec, tol in (("f64", 1e-13), ("f32", 1e-6)):
        U = f48.U64 if prec == "f64" else f48.U32
        out = h.dirac_apply(U, f48.pack(psi, prec, "odd"), m0, "fund", "hop_eo", dims, prec=prec)
        err = rel_err(f48.unpack(out, prec, "even"), oracle.hop_block(f48.U_orc, psi, 0))
        print(f"48^4 hop {prec}: {err:.3e}")
        assert err <= tol
        out = h.dirac_apply(U, f48.pack(psi, prec, "even"), m0, "fund", "eo", dims, prec=prec)
        err = rel_err(f48.unpack(out, prec, "even"), oracle.dhat(f48.U_orc, oracle.restrict(psi, 0), m0))
        print(f"48^4 dhat {prec}: {err:.3e}")
        assert err <= tol


def test_48_cg_both_modes(oracle, f48):
    h = hrd()
    dims, m0 = f48.dims, -0.3
    b = oracle.restrict(f48.spinor(4), 0)
    bp = f48.pack(b, "f64", "even")
    xs = {}
    for mode in ("f64", "mixed"):
        x, info = h.cg_solve(f48.U64, bp, m0, 1e-10, dims, "fund", mode=mode, U32=f48.U32)
        xe = f48.unpack(x, "f64", "even")
        res = oracle.true_residual(f48.U_orc, b, xe, m0)
        print(f"48^4 {mode}: {info} oracle residual {res:.3e}")
        assert res <= 1e-10
        xs[mode] = xe
    assert rel_err(xs["mixed"], xs["f64"]) < 1e-8


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
