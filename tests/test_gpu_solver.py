"""GPU parity of the level-1 linear algebra and of the CG solvers on D^+D^
(abstract: inverters; Sec. 2.1: the even/odd operator used in the HMC).

A solve is correct when the oracle, recomputing b - A x in FP64 from the
returned x, finds a relative residual <= tol (x is not unique to the bit);
x is also compared with the oracle's own CG solution.  Mixed precision must
reach the same true residual.  Error paths and determinism are checked
through the C ABI.
"""
import math

import numpy as np
import pytest
import torch

from gpu_util import Field, requires_gpu, rel_err, hrd

pytestmark = [pytest.mark.gpu, requires_gpu]


@pytest.fixture(scope="module")
def oracle():
    import oracle as O

    O._load()
    return O


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nparity", [1, 2])
def test_blas(prec, nparity):
    h = hrd()
    dims = (6, 4, 6, 10)
    F = Field(dims, "fund", seed=11)
    sites = "all" if nparity == 2 else "even"
    a_np, b_np = F.spinor(12), F.spinor(13)
    import oracle as O

    if nparity == 1:
        a_np, b_np = O.restrict(a_np, 0), O.restrict(b_np, 0)
    if prec == "f32":
        a_np = a_np.astype(np.complex64).astype(np.complex128)
        b_np = b_np.astype(np.complex64).astype(np.complex128)
    a = F.pack(a_np, prec, sites)
    b = F.pack(b_np, prec, sites)
    tol = 1e-13 if prec == "f64" else 1e-6
    dot = h.blas_dot(a, b, dims, "fund", prec, nparity)
    want = np.vdot(a_np.ravel(), b_np.ravel())
    assert abs(dot - want) <= 1e-13 * abs(want) * 10
    n2 = h.blas_norm2(a, dims, "fund", prec, nparity)
    assert abs(n2 - np.vdot(a_np.ravel(), a_np.ravel()).real) <= 1e-13 * n2
    # bitwise reproducible
    assert h.blas_dot(a, b, dims, "fund", prec, nparity) == dot
    c = complex(0.3, -1.7)
    nn = h.blas_axpy(c, a, b, dims, "fund", prec, nparity, norm=True)
    want_y = b_np + c * a_np
    got_y = F.unpack(b, prec, sites)
    assert rel_err(got_y, want_y) < tol
    assert abs(nn - np.vdot(got_y.ravel(), got_y.ravel()).real) <= 1e-12 * nn
    h.blas_xpay(a, c, b, dims, "fund", prec, nparity)
    want_y = a_np + c * got_y
    assert rel_err(F.unpack(b, prec, sites), want_y) < tol


CASES = [
    # (dims, rep, m0, kind, mode)
    ((8, 8, 8, 8), "fund", -0.2, "haar", "f64"),
    ((8, 8, 8, 8), "fund", -0.2, "haar", "mixed"),
    ((6, 4, 6, 10), "adj", -0.5, "haar", "f64"),
    ((6, 4, 6, 10), "adj", -0.5, "haar", "mixed"),
    ((8, 8, 8, 8), "fund", -0.3, "smeared", "mixed"),
    ((4, 4, 4, 4), "adj", -0.4, "haar", "mixed"),
]


@pytest.mark.parametrize("dims,rep,m0,kind,mode", CASES)
def test_cg_true_residual(oracle, dims, rep, m0, kind, mode):
    h = hrd()
    tol = 1e-10
    F = Field(dims, rep, seed=21, kind=kind)
    b_np = oracle.restrict(F.spinor(22), 0)
    b = F.pack(b_np, "f64", "even")
    x, info = h.cg_solve(F.U64, b, m0, tol, dims, rep, mode=mode, U32=F.U32)
    print(f"{dims} {rep} {mode}: {info}")
    xe = F.unpack(x, "f64", "even")
    res = oracle.true_residual(F.U_orc, b_np, xe, m0)
    assert res <= tol, res
    assert info["true_rel_residual"] <= tol
    assert abs(info["true_rel_residual"] - res) <= 1e-3 * tol + 0.05 * res
    if mode == "mixed":
        assert info["reliable_updates"] >= 1
    x_orc, oinfo = oracle.cg(F.U_orc, b_np, m0, tol=1e-12)
    err = rel_err(xe, x_orc)
    print(f"error vs FP64 oracle solution: {err:.3e} (oracle iters {oinfo['iters']})")
    assert err < 1e-7


def test_cg_warm_start_and_determinism(oracle):
    h = hrd()
    dims = (8, 8, 8, 8)
    F = Field(dims, "fund", seed=31)
    m0 = -0.2
    b_np = oracle.restrict(F.spinor(32), 0)
    b = F.pack(b_np, "f64", "even")
    x1, i1 = h.cg_solve(F.U64, b, m0, 1e-10, dims, "fund")
    x2, i2 = h.cg_solve(F.U64, b, m0, 1e-10, dims, "fund")
    assert torch.equal(x1, x2) and i1["iters"] == i2["iters"]
    x3, i3 = h.cg_solve(F.U64, b, m0, 1e-10, dims, "fund", mode="mixed", U32=F.U32)
    x4, i4 = h.cg_solve(F.U64, b, m0, 1e-10, dims, "fund", mode="mixed", U32=F.U32)
    assert torch.equal(x3, x4) and i3["iters"] == i4["iters"]
    # warm start from a converged solution: no iterations needed
    x5, i5 = h.cg_solve(F.U64, b, m0, 1e-10, dims, "fund", x0=x1)
    assert i5["iters"] == 0 and i5["true_rel_residual"] <= 1e-10


@pytest.mark.parametrize("mode", ["mixed", "mixed16"])
@pytest.mark.parametrize("delta", [0.1, 1e-8])
def test_mixed_cg_early_exit(oracle, mode, delta):
    """Mixed CG stopped after k iterations, on both sides of a wrap of the
    8-slot ring of search directions whose solution updates are deferred: the
    returned x must hold every direction's update.  FP32 inner operator: x is
    the oracle's k-th CG iterate up to FP32 rounding; F16: the true residual of
    x agrees with the iterated one (a missing update would leave the true
    residual at the size of an earlier iterate's)."""
    h = hrd()
    dims = (4, 4, 4, 8)
    m0 = -0.2
    F = Field(dims, "fund", seed=51, kind="smeared")
    U = F.U32 if mode == "mixed" else h.convert_gauge_prec(F.U64, dims, "fund", "f16")
    b_np = oracle.restrict(F.spinor(52), 0)
    b = F.pack(b_np, "f64", "even")
    for k in (1, 7, 8, 9, 16, 17):
        x, info = h.cg_solve(F.U64, b, m0, 1e-10, dims, "fund", mode=mode, U32=U, maxiter=k, delta=delta,
                             allow_noconv=True)
        assert info["status"] == "HRD_ENOCONV" and info["iters"] == k
        xe = F.unpack(x, "f64", "even")
        res = oracle.true_residual(F.U_orc, b_np, xe, m0)
        assert abs(info["true_rel_residual"] - res) <= 1e-6 * res
        it = info["iterated_rel_residual"]
        print(f"{mode} delta={delta} k={k}: true {res:.3e} iterated {it:.3e} updates {info['reliable_updates']}")
        if mode == "mixed":
            x_orc, _ = oracle.cg(F.U_orc, b_np, m0, tol=1e-30, maxiter=k)
            assert rel_err(xe, x_orc) < 1e-4, (k, rel_err(xe, x_orc))
        else:
            assert abs(res - it) <= 0.1 * it + 2e-3, (k, res, it)


@pytest.mark.parametrize("mode,delta", [("mixed", 1e-4), ("mixed16", 1e-4), ("mixed16", 1e-7)])
def test_mixed_cg_few_reliable_updates(oracle, mode, delta):
    """Small reliable-update thresholds: many passes through the ring of
    search directions between updates of the residual (and, for F16 fields,
    thresholds below the recurrence's drift, which the solver detects and
    raises); the true residual still reaches the tolerance."""
    h = hrd()
    dims = (8, 4, 4, 8)
    m0 = -0.3
    tol = 1e-10
    F = Field(dims, "adj", seed=61, kind="smeared")
    U = F.U32 if mode == "mixed" else h.convert_gauge_prec(F.U64, dims, "adj", "f16")
    b_np = oracle.restrict(F.spinor(62), 0)
    b = F.pack(b_np, "f64", "even")
    x, info = h.cg_solve(F.U64, b, m0, tol, dims, "adj", mode=mode, U32=U, delta=delta, maxiter=2000)
    print(f"{mode}: {info}")
    res = oracle.true_residual(F.U_orc, b_np, F.unpack(x, "f64", "even"), m0)
    assert res <= tol and info["iters"] > 24


@pytest.mark.parametrize("mode", ["f64", "mixed", "mixed16"])
def test_cg_on_side_stream(oracle, mode):
    """The solver works on the caller's stream (torch's current stream), including
    its pinned copies of the scalars and their events: the same solve on a second
    stream (default priority) gives the same x, bit for bit, and the same
    iteration count as on the default stream."""
    h = hrd()
    dims = (8, 4, 4, 8)
    F = Field(dims, "fund", seed=71, kind="smeared")
    U = {"f64": None, "mixed": F.U32, "mixed16": h.convert_gauge_prec(F.U64, dims, "fund", "f16")}[mode]
    b = F.pack(oracle.restrict(F.spinor(72), 0), "f64", "even")
    x0, i0 = h.cg_solve(F.U64, b, -0.3, 1e-10, dims, "fund", mode=mode, U32=U)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        x1, i1 = h.cg_solve(F.U64, b, -0.3, 1e-10, dims, "fund", mode=mode, U32=U)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert i1["iters"] == i0["iters"] and i1["reliable_updates"] == i0["reliable_updates"]
    assert torch.equal(x0, x1)
    assert oracle.true_residual(F.U_orc, oracle.restrict(F.spinor(72), 0), F.unpack(x1, "f64", "even"), -0.3) <= 1e-10


def test_cg_errors(oracle):
    h = hrd()
    dims = (4, 4, 4, 4)
    F = Field(dims, "fund", seed=41)
    b_np = oracle.restrict(F.spinor(42), 0)
    b = F.pack(b_np, "f64", "even")
    # maxiter too small -> ENOCONV with info filled
    x, info = h.cg_solve(F.U64, b, -0.2, 1e-10, dims, "fund", maxiter=2, allow_noconv=True)
    assert info["status"] == "HRD_ENOCONV" and info["iters"] == 2 and info["true_rel_residual"] > 1e-10
    with pytest.raises(h.HrdError) as e:
        h.cg_solve(F.U64, b, -0.2, 1e-10, dims, "fund", maxiter=2)
    assert e.value.status == h.ENOCONV
    # NaN source -> EBREAKDOWN
    bad = b_np.copy()
    bad.flat[5] = np.nan
    with pytest.raises(h.HrdError) as e:
        h.cg_solve(F.U64, F.pack(bad, "f64", "even"), -0.2, 1e-10, dims, "fund")
    assert e.value.status == h.EBREAKDOWN
    # tolerance below the FP64 floor -> ENOCONV with the achieved residual reported
    x, info = h.cg_solve(F.U64, b, -0.2, 1e-30, dims, "fund", maxiter=300, allow_noconv=True)
    assert info["status"] == "HRD_ENOCONV" and info["true_rel_residual"] < 1e-12
    # zero source -> x = 0
    z = F.pack(np.zeros_like(b_np), "f64", "even")
    x, info = h.cg_solve(F.U64, z, -0.2, 1e-10, dims, "fund")
    assert info["iters"] == 0 and float(x.abs().max()) == 0.0
    # mixed without FP32 links -> EINVAL
    with pytest.raises(h.HrdError) as e:
        h.cg_solve(F.U64, b, -0.2, 1e-10, dims, "fund", mode="mixed", U32=None)
    assert e.value.status == h.EINVAL


def test_abi_error_paths():
    import ctypes

    h = hrd()
    lib = h._lib
    bad = h.lattice((4, 4, 4, 5))
    assert lib.hrd_dirac_apply(ctypes.byref(bad), 0, 0, 1, 1, 2, 0.0, 0, 0, None, None) == h.ESHAPE
    assert "even" in lib.hrd_last_error().decode()
    lat = h.lattice((4, 4, 4, 4))
    assert lib.hrd_dirac_apply(ctypes.byref(lat), 11, 0, 1, 1, 2, 0.0, 0, 0, None, None) == h.EINVAL
    assert lib.hrd_dirac_apply(ctypes.byref(lat), 0, 0, None, 1, 2, 0.0, 0, 0, None, None) == h.EINVAL
    dims = (4, 4, 4, 4)
    F = Field(dims, "fund", seed=51)
    psi = F.pack(F.spinor(52), "f64", "all")
    with pytest.raises(h.HrdError) as e:
        h.dirac_apply(F.U64, psi, -0.2, "fund", "full", dims, out=psi)
    assert e.value.status == h.EALIAS
    with pytest.raises(h.HrdError) as e:
        h.dirac_apply(F.U64, psi, -4.0, "fund", "eo", dims)
    assert e.value.status == h.EINVAL
    assert lib.hrd_spinor_bytes(ctypes.byref(bad), 0, 0, 2) == 0
    assert lib.hrd_gauge_bytes(ctypes.byref(lat), 1, 1) == 256 * 4 * 36
