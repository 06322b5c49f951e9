"""Python binding of libhrd (ctypes): argument marshalling over the C ABI.

Every function takes and returns torch tensors on the GPU and forwards raw
device pointers, sizes and torch's current HIP stream to the library; no
computation happens here.  Packed fields are plain ``torch.uint8`` buffers
of the byte size the library reports (``spinor_bytes`` / ``gauge_bytes``);
natural-layout fields are complex128 (spinors [V, 4, N], gauge [4, V, 2, 2])
or float64 (adjoint gauge [4, V, 3, 3]) tensors, with V = T*L1*L2*L3 in
lexicographic site order.

The library is loaded from this directory; if it is missing the import
fails (build it with ``__graft_entry__.build()``): there is no CPU fallback.
"""
import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libhrd.so")

if not os.path.exists(LIBPATH):
    raise ImportError(f"libhrd.so not found at {LIBPATH}; build it with __graft_entry__.build()")

_lib = ctypes.CDLL(LIBPATH)
_lib.hrd_build_hash.restype = ctypes.c_char_p


def _check_build():
    from . import build as _build

    want = _build.source_hash()
    have = _lib.hrd_build_hash().decode()
    if have != want:
        raise ImportError(f"libhrd.so was built from other sources (library {have}, tree {want}); "
                          "rebuild it with __graft_entry__.build()")


_check_build()

# enums (hrd.h)
OK, EINVAL, ESHAPE, EALIAS, EHIP, ENOCONV, EBREAKDOWN, ESIZE = range(8)
FUND, ADJ, FUND_SU2, ADJ_SU2 = 0, 1, 2, 3
CPLX3, CPLX4, CPLX6, REAL8, SU3_ROW2, CPLX10, REAL15 = 4, 5, 6, 7, 8, 9, 10
SUN_FUND, SUN_ADJ, SUN_SYM, SUN_ASYM = 0, 1, 2, 3
F64, F32, F16 = 0, 1, 2
FULL, EO, HOP_EO, HOP_OE = 0, 1, 2, 3
SITES_ALL, SITES_EVEN, SITES_ODD = 0, 1, 2
CG_F64, CG_MIXED, CG_MIXED16 = 0, 1, 2

_STATUS_NAMES = {0: "HRD_OK", 1: "HRD_EINVAL", 2: "HRD_ESHAPE", 3: "HRD_EALIAS", 4: "HRD_EHIP",
                 5: "HRD_ENOCONV", 6: "HRD_EBREAKDOWN", 7: "HRD_ESIZE"}
_REPS = {"fund": FUND, "fundamental": FUND, "adj": ADJ, "adjoint": ADJ, "fund_su2": FUND_SU2,
         "adj_su2": ADJ_SU2, "cplx3": CPLX3, "cplx4": CPLX4, "cplx6": CPLX6, "real8": REAL8, "cplx10": CPLX10,
         "real15": REAL15,
         # SU(N > 2) representations by name -> their link formats
         "su3_fund": CPLX3, "su3_asym": CPLX3, "su3_sym": CPLX6, "su3_adj": REAL8, "su4_fund": CPLX4,
         "su4_asym": CPLX6, "su3_row2": SU3_ROW2, "su4_sym": CPLX10, "su4_adj": REAL15,
         FUND: FUND, ADJ: ADJ, FUND_SU2: FUND_SU2, ADJ_SU2: ADJ_SU2, CPLX3: CPLX3, CPLX4: CPLX4, CPLX6: CPLX6,
         REAL8: REAL8, SU3_ROW2: SU3_ROW2, CPLX10: CPLX10, REAL15: REAL15}
_SUN_KINDS = {"fund": SUN_FUND, "adj": SUN_ADJ, "sym": SUN_SYM, "asym": SUN_ASYM}
_PRECS = {"f64": F64, "fp64": F64, "f32": F32, "fp32": F32, "f16": F16, "fp16": F16, F64: F64, F32: F32,
          F16: F16, torch.float64: F64, torch.float32: F32}
_PARITIES = {"full": FULL, "eo": EO, "hop_eo": HOP_EO, "hop_oe": HOP_OE,
             FULL: FULL, EO: EO, HOP_EO: HOP_EO, HOP_OE: HOP_OE}
_SITES = {"all": SITES_ALL, "even": SITES_EVEN, "odd": SITES_ODD,
          SITES_ALL: SITES_ALL, SITES_EVEN: SITES_EVEN, SITES_ODD: SITES_ODD}
_MODES = {"f64": CG_F64, "fp64": CG_F64, "mixed": CG_MIXED, "mixed16": CG_MIXED16, CG_F64: CG_F64,
          CG_MIXED: CG_MIXED, CG_MIXED16: CG_MIXED16}


class HrdError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4)]


class CgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int), ("restarts", ctypes.c_int),
                ("true_rel_residual", ctypes.c_double), ("iterated_rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Problem(ctypes.Structure):
    _fields_ = [("lat", Lattice), ("rep", ctypes.c_int), ("nrhs", ctypes.c_int), ("m0", ctypes.c_double),
                ("U32", ctypes.c_void_p), ("U64", ctypes.c_void_p), ("src", ctypes.c_void_p),
                ("dst", ctypes.c_void_p)]


class Tune(ctypes.Structure):
    _fields_ = [("sites_per_tile", ctypes.c_int), ("rhs_per_tile", ctypes.c_int),
                ("block_threads", ctypes.c_int), ("blocks_per_cu", ctypes.c_int), ("slab_width", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_S = ctypes.c_size_t
_LP = ctypes.POINTER(Lattice)


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("hrd_last_error", ctypes.c_char_p)
_sig("hrd_version", ctypes.c_char_p)
_sig("hrd_spinor_bytes", _S, _LP, _I, _I, _I)
_sig("hrd_gauge_bytes", _S, _LP, _I, _I)
_sig("hrd_pack_gauge", _I, _LP, _I, _I, _P, _P, _P)
_sig("hrd_unpack_gauge", _I, _LP, _I, _I, _P, _P, _P)
_sig("hrd_represent", _I, _LP, _P, _P, _I, _P)
_sig("hrd_represent_backward", _I, _LP, _P, _P, _P, _P)
_sig("hrd_sun_rep_format", _I, _I, _I)
_sig("hrd_represent_sun", _I, _LP, _I, _I, _P, _P, _P)
_sig("hrd_represent_backward_sun", _I, _LP, _I, _I, _P, _P, _P, _P)
_sig("hrd_convert_gauge", _I, _LP, _I, _P, _P, _P)
_sig("hrd_pack_spinor", _I, _LP, _I, _I, _I, _P, _P, _P)
_sig("hrd_unpack_spinor", _I, _LP, _I, _I, _I, _P, _P, _P)
_sig("hrd_convert_spinor", _I, _LP, _I, _I, _I, _P, _P, _P)
_sig("hrd_convert_spinor_prec", _I, _LP, _I, _I, _I, _I, _P, _P, _P)
_sig("hrd_convert_gauge_prec", _I, _LP, _I, _I, _P, _P, _P)
_sig("hrd_dirac_workspace_bytes", _S, _LP, _I, _I, _I)
_sig("hrd_dirac_apply", _I, _LP, _I, _I, _P, _P, _P, _D, _I, _I, _P, _P)
_sig("hrd_blas_workspace_bytes", _S)
_sig("hrd_blas_dot", _I, _LP, _I, _I, _I, _P, _P, ctypes.POINTER(_D), _P, _P)
_sig("hrd_blas_norm2", _I, _LP, _I, _I, _I, _P, ctypes.POINTER(_D), _P, _P)
_sig("hrd_blas_axpy", _I, _LP, _I, _I, _I, _D, _D, _P, _P, ctypes.POINTER(_D), _P, _P)
_sig("hrd_blas_xpay", _I, _LP, _I, _I, _I, _P, _D, _D, _P, _P)
_sig("hrd_cg_workspace_bytes", _S, _LP, _I, _I)
_sig("hrd_cg_solve", _I, _LP, _I, _I, _P, _P, _P, _P, _D, _D, _I, _D, _P, _S, ctypes.POINTER(CgInfo), _P)
_sig("hrd_clover_bytes", _S, _LP, _I, _I)
_sig("hrd_clover_build", _I, _LP, _I, _I, _P, _D, _D, _P, _P, _P)
_sig("hrd_convert_clover", _I, _LP, _I, _P, _P, _P)
_sig("hrd_unpack_clover", _I, _LP, _I, _P, _P, _P)
_sig("hrd_dirac_apply_clover", _I, _LP, _I, _I, _P, _P, _P, _P, _P, _I, _I, _P, _P)
_sig("hrd_cg_solve_clover", _I, _LP, _I, _I, _P, _P, _P, _P, _P, _P, _P, _P, _D, _I, _D, _P, _S,
     ctypes.POINTER(CgInfo), _P)
_sig("hrd_dirac_force", _I, _LP, _I, _I, _P, _P, _P, _P, _D, _P)
_sig("hrd_action_force_workspace_bytes", _S, _LP, _I)
_sig("hrd_action_force", _I, _LP, _I, _P, _P, _P, _D, _D, _P, _S, _P)
_sig("hrd_stream_probe", _I, _P, _S, _P, _S, _I, _P)
_HAS_BATCHED = hasattr(_lib, "hrd_dirac_apply_batched")
if _HAS_BATCHED:
    _sig("hrd_batched_workspace_bytes", _S, ctypes.POINTER(Problem), _I, _I)
    _sig("hrd_dirac_apply_batched", _I, ctypes.POINTER(Problem), _I, _I, _I, ctypes.POINTER(Tune), _P, _S, _P)
    _sig("hrd_cg_batched_workspace_bytes", _S, ctypes.POINTER(Problem), _I)
    _sig("hrd_cg_solve_batched", _I, ctypes.POINTER(Problem), _I, _D, _I, _D, ctypes.POINTER(Tune), _P, _S,
         ctypes.POINTER(CgInfo), _P)
    _sig("hrd_autotune_batched", _I, ctypes.POINTER(Problem), _I, _P, _S, ctypes.c_char_p, ctypes.POINTER(Tune),
         _P)


def _check(status, allow=()):
    if status != OK and status not in allow:
        raise HrdError(status, _lib.hrd_last_error().decode())
    return status


def version():
    return _lib.hrd_version().decode()


def build_hash():
    """Hash of the sources the loaded library was built from (equal to the tree's)."""
    return _lib.hrd_build_hash().decode()


def lattice(dims):
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4:
        raise ValueError("dims must be (T, L1, L2, L3)")
    return Lattice((ctypes.c_int * 4)(*dims))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _need(t, nbytes, what):
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise ValueError(f"{what}: {have} bytes < required {nbytes}")


def _empty(nbytes, device=None):
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device or "cuda")


def _zeros(nbytes, device=None):
    return torch.zeros(int(nbytes), dtype=torch.uint8, device=device or "cuda")


@dataclass
class Geometry:
    dims: tuple
    rep: int

    @property
    def volume(self):
        T, a, b, c = self.dims
        return T * a * b * c

    @property
    def ncolour(self):
        return ncolour(self.rep)


def ncolour(rep):
    """Colours of the fermion in a link format (2, 3, 4, 6 or 8)."""
    return {FUND: 2, FUND_SU2: 2, ADJ: 3, ADJ_SU2: 3, CPLX3: 3, CPLX4: 4, CPLX6: 6, REAL8: 8, SU3_ROW2: 3,
            CPLX10: 10, REAL15: 15}[_REPS[rep]]


def base_rep(rep):
    """Uncompressed representation whose gauge layout derivatives use."""
    r = _REPS[rep]
    if r == SU3_ROW2:
        return CPLX3
    if r >= CPLX3:
        return r
    return FUND if ncolour(r) == 2 else ADJ


def spinor_bytes(dims, rep, prec, nparity):
    return _lib.hrd_spinor_bytes(ctypes.byref(lattice(dims)), _REPS[rep], _PRECS[prec], int(nparity))


def gauge_bytes(dims, rep, prec):
    return _lib.hrd_gauge_bytes(ctypes.byref(lattice(dims)), _REPS[rep], _PRECS[prec])


# ---------------------------------------------------------------------------
# gauge preparation
# ---------------------------------------------------------------------------

def pack_gauge(U_nat, dims, rep, prec):
    rep, prec = _REPS[rep], _PRECS[prec]
    out = _empty(gauge_bytes(dims, rep, prec), U_nat.device)
    _check(_lib.hrd_pack_gauge(ctypes.byref(lattice(dims)), rep, prec, _ptr(U_nat), _ptr(out), _stream()))
    return out


def unpack_gauge(U, dims, rep, prec):
    rep, prec = _REPS[rep], _PRECS[prec]
    V = Geometry(tuple(dims), rep).volume
    if rep in (ADJ, REAL8, REAL15):
        n = ncolour(rep)
        out = torch.empty((4, V, n, n), dtype=torch.float64, device=U.device)
    elif rep >= CPLX3:
        n = ncolour(rep)
        out = torch.empty((4, V, n, n), dtype=torch.complex128, device=U.device)
    else:
        out = torch.empty((4, V, 2, 2), dtype=torch.complex128, device=U.device)
    _check(_lib.hrd_unpack_gauge(ctypes.byref(lattice(dims)), rep, prec, _ptr(U), _ptr(out), _stream()))
    return out


def represent(U_fund, dims, prec=F64):
    prec = _PRECS[prec]
    out = _empty(gauge_bytes(dims, ADJ, prec), U_fund.device)
    _check(_lib.hrd_represent(ctypes.byref(lattice(dims)), _ptr(U_fund), _ptr(out), prec, _stream()))
    return out


def sun_rep_format(nc, kind):
    """Link format of representation kind ('fund', 'adj', 'sym', 'asym') of SU(nc), or None."""
    r = _lib.hrd_sun_rep_format(int(nc), _SUN_KINDS[kind])
    return None if r < 0 else r


def represent_sun(U_fund64, dims, nc, kind):
    """Packed FP64 links of representation kind of SU(nc) from the packed FP64
    fundamental field (format CPLX3 / CPLX4)."""
    fmt = sun_rep_format(nc, kind)
    if fmt is None:
        raise ValueError(f"no link format for SU({nc}) {kind}")
    out = _empty(gauge_bytes(dims, fmt, F64), U_fund64.device)
    _check(_lib.hrd_represent_sun(ctypes.byref(lattice(dims)), int(nc), _SUN_KINDS[kind], _ptr(U_fund64), _ptr(out),
                                  _stream()))
    return out


def represent_backward_sun(U_fund64, G_rep, dims, nc, kind):
    """Packed FP64 fundamental derivative (format CPLX3 / CPLX4) from a packed
    FP64 derivative with respect to the links of representation kind of SU(nc)
    (chain rule of represent_sun)."""
    fmt = sun_rep_format(nc, kind)
    if fmt is None:
        raise ValueError(f"no link format for SU({nc}) {kind}")
    _need(G_rep, gauge_bytes(dims, fmt, F64), "G_rep")
    out = _empty(gauge_bytes(dims, CPLX3 if nc == 3 else CPLX4, F64), U_fund64.device)
    _check(_lib.hrd_represent_backward_sun(ctypes.byref(lattice(dims)), int(nc), _SUN_KINDS[kind], _ptr(U_fund64),
                                           _ptr(G_rep), _ptr(out), _stream()))
    return out


def represent_backward(U_fund, g_adj, dims):
    out = _empty(gauge_bytes(dims, FUND, F64), U_fund.device)
    _check(_lib.hrd_represent_backward(ctypes.byref(lattice(dims)), _ptr(U_fund), _ptr(g_adj), _ptr(out), _stream()))
    return out


def convert_gauge(U64, dims, rep):
    rep = _REPS[rep]
    out = _empty(gauge_bytes(dims, rep, F32), U64.device)
    _check(_lib.hrd_convert_gauge(ctypes.byref(lattice(dims)), rep, _ptr(U64), _ptr(out), _stream()))
    return out


# ---------------------------------------------------------------------------
# spinors
# ---------------------------------------------------------------------------

def pack_spinor(psi_nat, dims, rep, prec, sites="all"):
    rep, prec, sites = _REPS[rep], _PRECS[prec], _SITES[sites]
    np_ = 2 if sites == SITES_ALL else 1
    out = _empty(spinor_bytes(dims, rep, prec, np_), psi_nat.device)
    _check(_lib.hrd_pack_spinor(ctypes.byref(lattice(dims)), rep, prec, sites, _ptr(psi_nat), _ptr(out), _stream()))
    return out


def unpack_spinor(psi, dims, rep, prec, sites="all", out=None):
    rep, prec, sites = _REPS[rep], _PRECS[prec], _SITES[sites]
    g = Geometry(tuple(dims), rep)
    if out is None:
        out = torch.zeros((g.volume, 4, g.ncolour), dtype=torch.complex128, device=psi.device)
    _check(_lib.hrd_unpack_spinor(ctypes.byref(lattice(dims)), rep, prec, sites, _ptr(psi), _ptr(out), _stream()))
    return out


def convert_spinor(psi, dims, rep, nparity, to_f32):
    rep = _REPS[rep]
    out = _empty(spinor_bytes(dims, rep, F32 if to_f32 else F64, nparity), psi.device)
    _check(_lib.hrd_convert_spinor(ctypes.byref(lattice(dims)), rep, int(nparity), int(bool(to_f32)), _ptr(psi),
                                   _ptr(out), _stream()))
    return out


def convert_spinor_prec(psi, dims, rep, nparity, prec_in, prec_out):
    """Packed spinor in prec_in -> new packed spinor in prec_out (F64, F32, F16)."""
    rep, pi, po = _REPS[rep], _PRECS[prec_in], _PRECS[prec_out]
    _need(psi, spinor_bytes(dims, rep, pi, nparity), "psi")
    out = _empty(spinor_bytes(dims, rep, po, nparity), psi.device)
    _check(_lib.hrd_convert_spinor_prec(ctypes.byref(lattice(dims)), rep, int(nparity), pi, po, _ptr(psi), _ptr(out),
                                        _stream()))
    return out


def convert_gauge_prec(U64, dims, rep, prec_out):
    """Packed FP64 gauge field -> packed F32 or F16 copy."""
    rep, po = _REPS[rep], _PRECS[prec_out]
    out = _empty(gauge_bytes(dims, rep, po), U64.device)
    _check(_lib.hrd_convert_gauge_prec(ctypes.byref(lattice(dims)), rep, po, _ptr(U64), _ptr(out), _stream()))
    return out


# ---------------------------------------------------------------------------
# operator
# ---------------------------------------------------------------------------

def dirac_workspace_bytes(dims, rep, prec, parity):
    return _lib.hrd_dirac_workspace_bytes(ctypes.byref(lattice(dims)), _REPS[rep], _PRECS[prec],
                                          _PARITIES[parity])


def dirac_apply(U, psi, m0, rep, parity, dims, prec=F64, dagger=False, out=None, work=None):
    """out = X psi for X in {D, D^, D_eo, D_oe} (parity 'full', 'eo', 'hop_eo', 'hop_oe')."""
    rep, prec, parity = _REPS[rep], _PRECS[prec], _PARITIES[parity]
    np_ = 2 if parity == FULL else 1
    nbytes = spinor_bytes(dims, rep, prec, np_)
    _need(psi, nbytes, "psi")
    _need(U, gauge_bytes(dims, rep, prec), "U")
    if out is None:
        out = _empty(nbytes, psi.device)
    wb = dirac_workspace_bytes(dims, rep, prec, parity)
    if wb and work is None:
        work = _empty(wb, psi.device)
    _check(_lib.hrd_dirac_apply(ctypes.byref(lattice(dims)), rep, prec, _ptr(U), _ptr(psi), _ptr(out), float(m0),
                                parity, int(bool(dagger)), _ptr(work) if wb else None, _stream()))
    return out


class DiracOp:
    """A prepared ``dirac_apply``: arguments are marshalled once, so repeated
    applications cost one foreign call each (used for timing loops and solvers
    written on top of the library).  The stream is torch's current stream at
    construction."""

    def __init__(self, U, dims, rep, prec, m0, parity, dagger=False):
        self.rep, self.prec, self.parity = _REPS[rep], _PRECS[prec], _PARITIES[parity]
        self.dims = tuple(dims)
        _need(U, gauge_bytes(dims, self.rep, self.prec), "U")
        self._U = U
        self._lat = lattice(dims)
        self._lat_ref = ctypes.byref(self._lat)
        np_ = 2 if self.parity == FULL else 1
        self.field_bytes = spinor_bytes(dims, self.rep, self.prec, np_)
        wb = dirac_workspace_bytes(dims, self.rep, self.prec, self.parity)
        self._work = _empty(wb, U.device) if wb else None
        self._wptr = self._work.data_ptr() if wb else None
        self._m0 = float(m0)
        self._dag = int(bool(dagger))
        self._stream = torch.cuda.current_stream().cuda_stream

    def __call__(self, src, dst):
        _need(src, self.field_bytes, "src")
        _need(dst, self.field_bytes, "dst")
        st = _lib.hrd_dirac_apply(self._lat_ref, self.rep, self.prec, self._U.data_ptr(), src.data_ptr(),
                                  dst.data_ptr(), self._m0, self.parity, self._dag, self._wptr, self._stream)
        if st != OK:
            _check(st)
        return dst


# ---------------------------------------------------------------------------
# level-1 linear algebra
# ---------------------------------------------------------------------------

_blas_work = {}


def _blas_ws(device):
    key = str(device)
    if key not in _blas_work:
        _blas_work[key] = _empty(_lib.hrd_blas_workspace_bytes(), device)
    return _blas_work[key]


def blas_dot(a, b, dims, rep, prec, nparity):
    res = (ctypes.c_double * 2)()
    _check(_lib.hrd_blas_dot(ctypes.byref(lattice(dims)), _REPS[rep], _PRECS[prec], int(nparity), _ptr(a), _ptr(b),
                             res, _ptr(_blas_ws(a.device)), _stream()))
    return complex(res[0], res[1])


def blas_norm2(a, dims, rep, prec, nparity):
    res = ctypes.c_double()
    _check(_lib.hrd_blas_norm2(ctypes.byref(lattice(dims)), _REPS[rep], _PRECS[prec], int(nparity), _ptr(a),
                               ctypes.byref(res), _ptr(_blas_ws(a.device)), _stream()))
    return res.value


def blas_axpy(a, x, y, dims, rep, prec, nparity, norm=False):
    a = complex(a)
    res = ctypes.c_double()
    _check(_lib.hrd_blas_axpy(ctypes.byref(lattice(dims)), _REPS[rep], _PRECS[prec], int(nparity), a.real, a.imag,
                              _ptr(x), _ptr(y), ctypes.byref(res) if norm else None, _ptr(_blas_ws(x.device)),
                              _stream()))
    return res.value if norm else None


def blas_xpay(x, a, y, dims, rep, prec, nparity):
    a = complex(a)
    _check(_lib.hrd_blas_xpay(ctypes.byref(lattice(dims)), _REPS[rep], _PRECS[prec], int(nparity), _ptr(x), a.real,
                              a.imag, _ptr(y), _stream()))


# ---------------------------------------------------------------------------
# solvers
# ---------------------------------------------------------------------------

def cg_workspace_bytes(dims, rep, mode):
    return _lib.hrd_cg_workspace_bytes(ctypes.byref(lattice(dims)), _REPS[rep], _MODES[mode])


def cg_solve(U64, b, m0, tol, dims, rep, mode="f64", U32=None, x0=None, maxiter=10000, delta=0.0, work=None,
             allow_noconv=False):
    """Solve (D^+ D^) x = b on even sites; returns (x, info dict).  U32 is the
    reduced-precision gauge copy: FP32 for mode 'mixed', F16 for 'mixed16'.
    delta is the reliable-update threshold (0: the library's default for the
    mode)."""
    rep, mode = _REPS[rep], _MODES[mode]
    nb = spinor_bytes(dims, rep, F64, 1)
    _need(b, nb, "b")
    x = _zeros(nb, b.device) if x0 is None else x0.clone()
    wb = cg_workspace_bytes(dims, rep, mode)
    if work is None:
        work = _empty(wb, b.device)
    info = CgInfo()
    st = _lib.hrd_cg_solve(ctypes.byref(lattice(dims)), rep, mode, _ptr(U64), _ptr(U32), _ptr(b), _ptr(x), float(m0),
                           float(tol), int(maxiter), float(delta), _ptr(work), wb, ctypes.byref(info), _stream())
    _check(st, allow=(ENOCONV,) if allow_noconv else ())
    d = info.as_dict()
    d["status"] = _STATUS_NAMES[st]
    return x, d


# ---------------------------------------------------------------------------
# clover term
# ---------------------------------------------------------------------------

def clover_bytes(dims, rep, prec):
    return _lib.hrd_clover_bytes(ctypes.byref(lattice(dims)), _REPS[rep], _PRECS[prec])


@dataclass
class Clover:
    """Packed clover fields M = m + A and M^{-1} of one precision."""
    M: torch.Tensor
    Minv: torch.Tensor
    prec: int


CLOVER_SW, CLOVER_EXP = 0, 1
_CLOVER_KINDS = {"sw": CLOVER_SW, "exp": CLOVER_EXP, CLOVER_SW: CLOVER_SW, CLOVER_EXP: CLOVER_EXP}


def clover_build(U64, csw, m0, dims, rep, kind="sw"):
    """FP64 M and M^{-1} from the packed FP64 gauge field: kind 'sw' builds
    M = (4 + m0) + A, kind 'exp' builds M = m exp(A/m)."""
    rep = _REPS[rep]
    nb = clover_bytes(dims, rep, F64)
    _need(U64, gauge_bytes(dims, rep, F64), "U64")
    M, Minv = _empty(nb, U64.device), _empty(nb, U64.device)
    _check(_lib.hrd_clover_build(ctypes.byref(lattice(dims)), rep, _CLOVER_KINDS[kind], _ptr(U64), float(csw),
                                 float(m0), _ptr(M), _ptr(Minv), _stream()))
    return Clover(M, Minv, F64)


def convert_clover(c64, dims, rep):
    """FP32 copy of an FP64 Clover pair."""
    rep = _REPS[rep]
    nb = clover_bytes(dims, rep, F32)
    out = []
    for t in (c64.M, c64.Minv):
        o = _empty(nb, t.device)
        _check(_lib.hrd_convert_clover(ctypes.byref(lattice(dims)), rep, _ptr(t), _ptr(o), _stream()))
        out.append(o)
    return Clover(out[0], out[1], F32)


def unpack_clover(C64, dims, rep):
    """Packed FP64 clover field -> complex128 [V, 4N, 4N]."""
    rep = _REPS[rep]
    g = Geometry(tuple(dims), rep)
    _need(C64, clover_bytes(dims, rep, F64), "C64")
    n = 4 * g.ncolour
    out = torch.empty((g.volume, n, n), dtype=torch.complex128, device=C64.device)
    _check(_lib.hrd_unpack_clover(ctypes.byref(lattice(dims)), rep, _ptr(C64), _ptr(out), _stream()))
    return out


def dirac_apply_clover(U, clov, psi, rep, parity, dims, dagger=False, out=None, work=None, prec=None):
    """out = D_sw psi ('full') or D^_sw psi_e ('eo'); the precision is that of
    clov unless prec = 'f16' is given (F16 fields with FP32 clover fields)."""
    rep, parity = _REPS[rep], _PARITIES[parity]
    prec = clov.prec if prec is None else _PRECS[prec]
    np_ = 2 if parity == FULL else 1
    nbytes = spinor_bytes(dims, rep, prec, np_)
    _need(psi, nbytes, "psi")
    _need(U, gauge_bytes(dims, rep, prec), "U")
    if out is None:
        out = _empty(nbytes, psi.device)
    wb = dirac_workspace_bytes(dims, rep, prec, parity)
    if wb and work is None:
        work = _empty(wb, psi.device)
    _check(_lib.hrd_dirac_apply_clover(ctypes.byref(lattice(dims)), rep, prec, _ptr(U), _ptr(clov.M),
                                       _ptr(clov.Minv), _ptr(psi), _ptr(out), parity, int(bool(dagger)),
                                       _ptr(work) if wb else None, _stream()))
    return out


class CloverOp:
    """Prepared ``dirac_apply_clover`` (one foreign call per application)."""

    def __init__(self, U, clov, dims, rep, parity, dagger=False, prec=None):
        self.rep, self.parity = _REPS[rep], _PARITIES[parity]
        self.prec = clov.prec if prec is None else _PRECS[prec]
        _need(U, gauge_bytes(dims, self.rep, self.prec), "U")
        self._keep = (U, clov)
        self._lat = lattice(dims)
        self._lat_ref = ctypes.byref(self._lat)
        np_ = 2 if self.parity == FULL else 1
        self.field_bytes = spinor_bytes(dims, self.rep, self.prec, np_)
        wb = dirac_workspace_bytes(dims, self.rep, self.prec, self.parity)
        self._work = _empty(wb, U.device) if wb else None
        self._args = (U.data_ptr(), clov.M.data_ptr(), clov.Minv.data_ptr())
        self._wptr = self._work.data_ptr() if wb else None
        self._dag = int(bool(dagger))
        self._stream = torch.cuda.current_stream().cuda_stream

    def __call__(self, src, dst):
        _need(src, self.field_bytes, "src")
        _need(dst, self.field_bytes, "dst")
        st = _lib.hrd_dirac_apply_clover(self._lat_ref, self.rep, self.prec, *self._args, src.data_ptr(),
                                         dst.data_ptr(), self.parity, self._dag, self._wptr, self._stream)
        if st != OK:
            _check(st)
        return dst


def cg_solve_clover(U64, clov64, b, tol, dims, rep, mode="f64", U32=None, clov32=None, x0=None, maxiter=10000,
                    delta=0.0, work=None, allow_noconv=False):
    """Solve (D^_sw^+ D^_sw) x = b on even sites; returns (x, info dict)."""
    rep, mode = _REPS[rep], _MODES[mode]
    nb = spinor_bytes(dims, rep, F64, 1)
    _need(b, nb, "b")
    x = _zeros(nb, b.device) if x0 is None else x0.clone()
    wb = cg_workspace_bytes(dims, rep, mode)
    if work is None:
        work = _empty(wb, b.device)
    info = CgInfo()
    M32 = clov32.M if clov32 is not None else None
    Mi32 = clov32.Minv if clov32 is not None else None
    st = _lib.hrd_cg_solve_clover(ctypes.byref(lattice(dims)), rep, mode, _ptr(U64), _ptr(U32), _ptr(clov64.M),
                                  _ptr(clov64.Minv), _ptr(M32), _ptr(Mi32), _ptr(b), _ptr(x), float(tol),
                                  int(maxiter), float(delta), _ptr(work), wb, ctypes.byref(info), _stream())
    _check(st, allow=(ENOCONV,) if allow_noconv else ())
    d = info.as_dict()
    d["status"] = _STATUS_NAMES[st]
    return x, d


# ---------------------------------------------------------------------------
# force
# ---------------------------------------------------------------------------

def dirac_force(U, X, Y, dims, rep, scale=1.0, prec=F64):
    """F = scale * d/dU Re<X, D[U] Y> (packed FP64 gauge layout)."""
    rep = _REPS[rep]
    out = _empty(gauge_bytes(dims, base_rep(rep), F64), X.device)
    _check(_lib.hrd_dirac_force(ctypes.byref(lattice(dims)), rep, _PRECS[prec], _ptr(U), _ptr(X), _ptr(Y), _ptr(out),
                                float(scale), _stream()))
    return out


def action_force(U, xi, m0, dims, rep, scale=1.0):
    """scale * dS/dU for S = phi^+ (D^+ D^)^{-1} phi, given xi = (D^+ D^)^{-1} phi."""
    rep = _REPS[rep]
    out = _empty(gauge_bytes(dims, base_rep(rep), F64), xi.device)
    wb = _lib.hrd_action_force_workspace_bytes(ctypes.byref(lattice(dims)), rep)
    work = _empty(wb, xi.device)
    _check(_lib.hrd_action_force(ctypes.byref(lattice(dims)), rep, _ptr(U), _ptr(xi), _ptr(out), float(m0),
                                 float(scale), _ptr(work), wb, _stream()))
    return out


# ---------------------------------------------------------------------------
# batched
# ---------------------------------------------------------------------------

def has_batched():
    return _HAS_BATCHED


def make_problems(specs):
    """specs: list of dicts with dims, rep, nrhs, m0, U32, U64, src, dst (tensors or None)."""
    arr = (Problem * len(specs))()
    for i, s in enumerate(specs):
        arr[i].lat = lattice(s["dims"])
        arr[i].rep = _REPS[s["rep"]]
        arr[i].nrhs = int(s["nrhs"])
        arr[i].m0 = float(s["m0"])
        arr[i].U32 = s["U32"].data_ptr() if s.get("U32") is not None else None
        arr[i].U64 = s["U64"].data_ptr() if s.get("U64") is not None else None
        arr[i].src = s["src"].data_ptr() if s.get("src") is not None else None
        arr[i].dst = s["dst"].data_ptr() if s.get("dst") is not None else None
    return arr


def _tune_ptr(tune):
    if tune is None:
        return None
    if isinstance(tune, dict):
        t = Tune(**tune)
    else:
        t = tune
    return ctypes.byref(t)


def batched_workspace_bytes(problems, parity):
    return _lib.hrd_batched_workspace_bytes(problems, len(problems), _PARITIES[parity])


def dirac_apply_batched(problems, parity, dagger=False, tune=None, work=None, device="cuda"):
    wb = batched_workspace_bytes(problems, parity)
    if work is None:
        work = _empty(max(wb, 1), device)
    _check(_lib.hrd_dirac_apply_batched(problems, len(problems), _PARITIES[parity], int(bool(dagger)),
                                        _tune_ptr(tune), _ptr(work), wb, _stream()))


def cg_solve_batched(problems, tol, maxiter=10000, delta=0.0, tune=None, work=None, device="cuda",
                     allow_noconv=False):
    wb = _lib.hrd_cg_batched_workspace_bytes(problems, len(problems))
    if work is None:
        work = _empty(wb, device)
    ntot = sum(p.nrhs for p in problems)
    infos = (CgInfo * ntot)()
    st = _lib.hrd_cg_solve_batched(problems, len(problems), float(tol), int(maxiter), float(delta), _tune_ptr(tune),
                                   _ptr(work), wb, infos, _stream())
    _check(st, allow=(ENOCONV,) if allow_noconv else ())
    return [i.as_dict() for i in infos], _STATUS_NAMES[st]


def autotune_batched(problems, cache_path=None, work=None, device="cuda"):
    wb = batched_workspace_bytes(problems, EO)
    if work is None:
        work = _empty(wb, device)
    best = Tune()
    _check(_lib.hrd_autotune_batched(problems, len(problems), _ptr(work), wb,
                                     cache_path.encode() if cache_path else None, ctypes.byref(best), _stream()))
    return best.as_dict()


# ---------------------------------------------------------------------------
# bandwidth ceiling
# ---------------------------------------------------------------------------

def stream_probe(src, dst, read_bytes, write_bytes, tiled=True):
    """Stream read_bytes of src and write write_bytes of dst (k = read/write
    16-byte loads per store) with the operator kernels' access instructions;
    asynchronous on torch's current stream."""
    _need(src, read_bytes, "stream_probe src")
    _need(dst, write_bytes, "stream_probe dst")
    _check(_lib.hrd_stream_probe(_ptr(src), int(read_bytes), _ptr(dst), int(write_bytes), int(bool(tiled)),
                                 _stream()))
