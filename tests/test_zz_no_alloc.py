"""hrd_dirac_apply_static — the entry point for callers that cannot allocate
(odd temporary of the even/odd operator in a static device array) — returns
what hrd_dirac_apply with a caller workspace returns, bit for bit, through the
C ABI, on consecutive calls of decreasing size, and refuses a temporary beyond
its static size before touching the device."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2411_18511_amd import hrd, inputs

pytestmark = pytest.mark.gpu


def _fn():
    f = hrd._lib.hrd_dirac_apply_static
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.POINTER(hrd.Lattice), ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    return f


def _fields(dims, rep, prec, seed):
    V = int(np.prod(dims))
    Uf = torch.from_numpy(inputs.gauge_field(dims, seed).reshape(4, V, 2, 2)).cuda()
    U64 = hrd.pack_gauge(Uf, dims, "fund", "f64")
    if rep == "adj":
        U64 = hrd.represent(U64, dims, "f64")
    U = U64 if prec == "f64" else hrd.convert_gauge_prec(U64, dims, rep, prec)
    n = 2 if rep == "fund" else 3
    psi = torch.from_numpy(inputs.gaussian_spinor(dims, n, seed + 1).reshape(V, 4, n)).cuda()
    return U, {s: hrd.convert_spinor_prec(hrd.pack_spinor(psi, dims, rep, "f64", s), dims, rep,
                                          2 if s == "all" else 1, "f64", prec) if prec != "f64"
               else hrd.pack_spinor(psi, dims, rep, "f64", s) for s in ("all", "even", "odd")}


@pytest.mark.parametrize("rep,prec", [("fund", "f64"), ("fund", "f32"), ("fund", "f16"), ("adj", "f64")])
def test_static_equals_workspace_entry_point(rep, prec):
    f = _fn()
    m0 = -0.3
    for dims in ((8, 8, 8, 8), (4, 4, 4, 6)):  # the second call is smaller than the first
        U, src = _fields(dims, rep, prec, 7)
        lat = hrd.lattice(dims)
        for parity, sname in (("eo", "even"), ("hop_eo", "odd"), ("full", "all")):
            for dagger in (False, True):
                want = hrd.dirac_apply(U, src[sname], m0, rep, parity, dims, prec=prec, dagger=dagger)
                got = torch.full_like(want, 0x5A)
                st = f(ctypes.byref(lat), hrd._REPS[rep], hrd._PRECS[prec], U.data_ptr(), src[sname].data_ptr(),
                       got.data_ptr(), m0, hrd._PARITIES[parity], int(dagger),
                       torch.cuda.current_stream().cuda_stream)
                assert st == hrd.OK, hrd._lib.hrd_last_error()
                torch.cuda.synchronize()
                assert torch.equal(got, want), (dims, parity, dagger)


def test_static_scratch_limit():
    f = _fn()
    hrd._lib.hrd_dirac_static_scratch_bytes.restype = ctypes.c_size_t
    cap = hrd._lib.hrd_dirac_static_scratch_bytes()
    assert cap == 64 << 20
    # 32^4 adjoint FP64: the odd temporary is 524288 sites x 192 B = 96 MiB > 64 MiB
    dims = (32, 32, 32, 32)
    assert hrd.spinor_bytes(dims, "adj", "f64", 1) > cap
    st = f(ctypes.byref(hrd.lattice(dims)), hrd.ADJ, hrd.F64, None, None, None, -0.3, hrd.EO, 0, None)
    assert st == hrd.ESIZE
    assert b"static scratch" in hrd._lib.hrd_last_error()
    # the largest accepted size: 32^4 fundamental FP64 (524288 x 128 B = 64 MiB) passes the size check and
    # then fails on the NULL fields, before any launch
    st = f(ctypes.byref(hrd.lattice(dims)), hrd.FUND, hrd.F64, None, None, None, -0.3, hrd.EO, 0, None)
    assert st == hrd.EINVAL
