"""Oracle — TEST INFRASTRUCTURE ONLY.

Plain FP64 CPU definitions of everything the GPU library computes, for SU(2)
Wilson fermions in the fundamental and adjoint representations.  Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import
this package; the GPU library never does, and the two share no code.

The paper (arXiv:2411.18511) reports the performance of the unimproved
Wilson-Dirac operator (Sec. 2.1, Table 1), its even/odd preconditioned form
used inside HMC (Sec. 2.1), fermions in the fundamental and higher
representations (Sec. 1) and "a range of inverters" (abstract), without
writing any of them down.  The readings taken here are standard lattice field
theory; the C part (``oracle.c``) states the operator conventions in its
header.  Additional readings fixed in this module:

* Even/odd: parity(x) = (t + x1 + x2 + x3) mod 2, even = 0.  With m = 4 + m0,
  D = [[m, D_eo], [D_oe, m]] in (even, odd) blocks, D_eo = -H_eo / 2, and the
  preconditioned operator on even sites is the Schur complement
  D^ = m - (1/m) D_eo D_oe (Sec. 2.1, "even-odd preconditioned version").
* Daggers use gamma5-hermiticity, D^+ = g5 D g5 (g5 = g0 g1 g2 g3).
* The solver is conjugate gradients (Hestenes-Stiefel) on A = D^+ D^ over
  even sites, from x0 = 0, with residual ||b - A x|| / ||b|| (not squared).
* Adjoint representation R_ab(U) = tr(s_a U s_b U^+) / 2 (real 3x3).
* Force: G = dL/dRe U + i dL/dIm U for L = Re<X, D[U] Y>; for the real
  adjoint links the derivative is Re G.
* Fermion action S = phi^+ A^{-1} phi on even sites; dS/dU = (2/m) G[X, Y]
  with xi = A^{-1} phi, eta = D^ xi, Y = (xi, D_oe xi), X = (eta, D_eo^+ eta).

Field layouts are natural: gauge [4, T, L1, L2, L3, N, N], spinor
[T, L1, L2, L3, 4, N] (spin-major, then colour).  Even-site fields are stored
as full-lattice arrays whose odd sites are zero.
"""
import ctypes
import os
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b

            _b.build()
        lib = ctypes.CDLL(_LIBPATH)
        P = ctypes.c_void_p
        lib.oracle_gamma.argtypes = [ctypes.c_int, P]
        lib.oracle_hopping.argtypes = [P, ctypes.c_int, P, P, P, ctypes.c_int]
        lib.oracle_dirac.argtypes = [P, ctypes.c_int, P, P, P, ctypes.c_double]
        lib.oracle_represent_adjoint.argtypes = [ctypes.c_long, P, P]
        lib.oracle_force.argtypes = [P, ctypes.c_int, P, P, P]
        lib.oracle_plaquette.argtypes = [P, ctypes.c_int, P]
        lib.oracle_plaquette.restype = ctypes.c_double
        lib.oracle_clover.argtypes = [P, ctypes.c_int, P, ctypes.c_double, P]
        lib.oracle_cg.argtypes = [P, ctypes.c_int, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        lib.oracle_cg.restype = ctypes.c_int
        lib.oracle_true_residual.argtypes = [P, ctypes.c_int, P, P, P, ctypes.c_double]
        lib.oracle_true_residual.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims_arr(dims):
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int32))


def _cplx(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _dims_of_spinor(psi):
    return tuple(psi.shape[:4])


# ---------------------------------------------------------------------------
# Basic objects
# ---------------------------------------------------------------------------

def gamma(mu):
    """Euclidean gamma matrix g_mu of the chiral basis (4x4 complex)."""
    out = np.zeros((4, 4), np.complex128)
    _load().oracle_gamma(int(mu), _ptr(out))
    return out


def gamma5():
    """g5 = g0 g1 g2 g3."""
    return gamma(0) @ gamma(1) @ gamma(2) @ gamma(3)


def apply_gamma5(psi):
    """Multiply every site's spinor by g5 (acts on the spin index)."""
    return np.einsum("ab,...bi->...ai", gamma5(), psi)


def parity(dims):
    """Array of site parities (t + x1 + x2 + x3) mod 2, shape dims."""
    t, x1, x2, x3 = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    return (t + x1 + x2 + x3) % 2


def restrict(psi, par):
    """Copy of psi with the sites of the other parity set to zero."""
    mask = parity(_dims_of_spinor(psi)) == par
    return psi * mask[..., None, None]


def inner(a, b):
    """<a, b> = sum conj(a) b."""
    return np.vdot(a.ravel(), b.ravel())


def norm(a):
    return float(np.sqrt(np.real(inner(a, a))))


def _links_complex(U):
    return _cplx(U)


# ---------------------------------------------------------------------------
# Operators
# ---------------------------------------------------------------------------

def hopping(U, psi, mask=3):
    """(H psi) on the sites whose parity bit is in mask (1 even, 2 odd, 3 all)."""
    dims = _dims_of_spinor(psi)
    n = psi.shape[-1]
    psi = _cplx(psi)
    out = np.empty_like(psi)
    _load().oracle_hopping(_ptr(_dims_arr(dims)), n, _ptr(_links_complex(U)), _ptr(psi),
                           _ptr(out), int(mask))
    return out


def dirac(U, psi, m0):
    """D psi = (4 + m0) psi - H psi / 2 on the whole lattice."""
    dims = _dims_of_spinor(psi)
    n = psi.shape[-1]
    psi = _cplx(psi)
    out = np.empty_like(psi)
    _load().oracle_dirac(_ptr(_dims_arr(dims)), n, _ptr(_links_complex(U)), _ptr(psi),
                         _ptr(out), float(m0))
    return out


def dirac_dagger(U, psi, m0):
    """D^+ psi = g5 D g5 psi."""
    return apply_gamma5(dirac(U, apply_gamma5(psi), m0))


def hop_block(U, psi, target):
    """Off-diagonal block of D: D_eo psi_o (target=0) or D_oe psi_e (target=1).

    Reads psi on the sites of parity 1 - target only; returns a field that is
    zero off the target parity.
    """
    src = restrict(psi, 1 - target)
    return -0.5 * hopping(U, src, 1 << target)


def hop_block_dagger(U, psi, target):
    """(D_{1-target, target})^+ psi = g5 D_{target,1-target} g5 psi."""
    return apply_gamma5(hop_block(U, apply_gamma5(psi), target))


def dhat(U, psi_e, m0):
    """Even/odd preconditioned operator D^ psi_e = m psi_e - (1/m) D_eo D_oe psi_e."""
    m = 4.0 + m0
    psi_e = restrict(psi_e, 0)
    t_o = hop_block(U, psi_e, 1)
    return m * psi_e - hop_block(U, t_o, 0) / m


def dhat_dagger(U, psi_e, m0):
    return apply_gamma5(dhat(U, apply_gamma5(psi_e), m0))


def normal_op(U, x_e, m0):
    """A x = D^+ D^ x on even sites."""
    return dhat_dagger(U, dhat(U, x_e, m0), m0)


def cg(U, b_e, m0, tol=1e-10, maxiter=10000, x0=None, op=None):
    """Conjugate gradients for (D^+ D^) x = b on even sites.

    Plain Hestenes-Stiefel iteration; stops when the recursively updated
    residual satisfies ||r|| <= tol ||b||, then recomputes the true residual
    b - A x and continues from it if that check fails.  Returns (x, info).
    `op(x)` replaces D^+ D^ x when given (e.g. the clover operator).
    """
    if op is None:
        def op(v):
            return normal_op(U, v, m0)
    b_e = restrict(_cplx(b_e), 0)
    bnorm = norm(b_e)
    x = np.zeros_like(b_e) if x0 is None else restrict(_cplx(x0), 0)
    r = b_e - op(x) if x0 is not None else b_e.copy()
    p = r.copy()
    rr = np.real(inner(r, r))
    iters = 0
    t0 = time.perf_counter()
    while iters < maxiter:
        if np.sqrt(rr) <= tol * bnorm:
            r_true = b_e - op(x)
            rr_true = np.real(inner(r_true, r_true))
            if np.sqrt(rr_true) <= tol * bnorm:
                break
            r = r_true
            p = r.copy()
            rr = rr_true
        Ap = op(p)
        alpha = rr / np.real(inner(p, Ap))
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = np.real(inner(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        iters += 1
    res = norm(b_e - op(x)) / bnorm
    return x, {"iters": iters, "true_rel_residual": res, "seconds": time.perf_counter() - t0}


def cg_native(U, b_e, m0, tol=1e-10, maxiter=10000, progress=0):
    """The iteration of cg() (x0 = 0, default operator) run entirely in the C
    part, for lattices where the numpy version is too slow.  Returns (x, info)
    like cg(); progress > 0 prints the residual every `progress` iterations."""
    dims = _dims_of_spinor(b_e)
    n = b_e.shape[-1]
    b = _cplx(b_e)
    x = np.empty_like(b)
    res = ctypes.c_double(0.0)
    t0 = time.perf_counter()
    it = _load().oracle_cg(_ptr(_dims_arr(dims)), n, _ptr(_links_complex(U)), _ptr(b), _ptr(x), float(m0),
                           float(tol), int(maxiter), ctypes.byref(res), int(progress))
    if it < 0:
        raise MemoryError("oracle_cg: temporaries could not be allocated")
    return x, {"iters": it, "true_rel_residual": res.value, "seconds": time.perf_counter() - t0}


def true_residual_native(U, b_e, x_e, m0):
    """true_residual() evaluated in the C part (same operator as cg_native)."""
    dims = _dims_of_spinor(b_e)
    n = b_e.shape[-1]
    res = _load().oracle_true_residual(_ptr(_dims_arr(dims)), n, _ptr(_links_complex(U)), _ptr(_cplx(b_e)),
                                       _ptr(_cplx(x_e)), float(m0))
    if res < 0:
        raise MemoryError("oracle_true_residual: temporaries could not be allocated")
    return res


def true_residual(U, b_e, x_e, m0):
    """||b - D^+ D^ x|| / ||b|| on even sites."""
    b_e = restrict(_cplx(b_e), 0)
    return norm(b_e - normal_op(U, restrict(_cplx(x_e), 0), m0)) / norm(b_e)


# ---------------------------------------------------------------------------
# Gauge-field maps
# ---------------------------------------------------------------------------

def represent_adjoint(Uf):
    """R_ab(U) = tr(s_a U s_b U^+) / 2 for every link; real, shape [..., 3, 3]."""
    Uf = _cplx(Uf)
    shape = Uf.shape[:-2]
    nl = int(np.prod(shape))
    R = np.empty(shape + (3, 3), np.float64)
    _load().oracle_represent_adjoint(nl, _ptr(Uf), _ptr(R))
    return R


def plaquette(U):
    """Average plaquette (1/N) Re tr of the elementary loop, over sites and planes."""
    n = U.shape[-1]
    dims = U.shape[1:5]
    return _load().oracle_plaquette(_ptr(_dims_arr(dims)), n, _ptr(_links_complex(U)))


# ---------------------------------------------------------------------------
# Derivatives
# ---------------------------------------------------------------------------

def force(X, Y, real_links=False):
    """G = dL/dRe U + i dL/dIm U for L = Re<X, D[U] Y>; shape [4, T, L1, L2, L3, N, N].

    For real (adjoint) links the derivative with respect to the real entries
    is Re G, returned when real_links is true.
    """
    dims = _dims_of_spinor(X)
    n = X.shape[-1]
    X = _cplx(X)
    Y = _cplx(Y)
    G = np.empty((4,) + tuple(dims) + (n, n), np.complex128)
    _load().oracle_force(_ptr(_dims_arr(dims)), n, _ptr(X), _ptr(Y), _ptr(G))
    return G.real.copy() if real_links else G


def action_force_fields(U, xi_e, m0):
    """The (X, Y) pair whose force gives dS/dU = (2/m) G[X, Y] for S = phi^+ A^{-1} phi.

    xi_e = A^{-1} phi; eta = D^ xi; Y = (xi on even, D_oe xi on odd);
    X = (eta on even, D_eo^+ eta on odd).
    """
    xi_e = restrict(_cplx(xi_e), 0)
    eta = dhat(U, xi_e, m0)
    Y = xi_e + hop_block(U, xi_e, 1)
    X = eta + hop_block_dagger(U, eta, 1)
    return X, Y


def action_force(U, phi_e, m0, tol=1e-12, maxiter=10000, real_links=False):
    """dS/dU for S = Re<phi, A^{-1} phi>, A = D^+ D^ (solve by cg)."""
    xi, info = cg(U, phi_e, m0, tol=tol, maxiter=maxiter)
    X, Y = action_force_fields(U, xi, m0)
    m = 4.0 + m0
    return (2.0 / m) * force(X, Y, real_links=real_links), xi, info


# ---------------------------------------------------------------------------
# Clover (Sheikholeslami-Wohlert) term — the paper's Sec. 2.2 diagonal term
# ---------------------------------------------------------------------------

def clover(U, csw):
    """A(x) = c_sw (i/4) sum_{mu,nu} sigma_{mu nu} (x) F_{mu nu}(x) for every site;
    shape [T, L1, L2, L3, 4N, 4N] (row index spin * N + colour).  See oracle.c."""
    dims = U.shape[1:5]
    n = U.shape[-1]
    A = np.empty(tuple(dims) + (4 * n, 4 * n), np.complex128)
    _load().oracle_clover(_ptr(_dims_arr(dims)), n, _ptr(_links_complex(U)), float(csw), _ptr(A))
    return A


def apply_site_matrix(M, psi):
    """(M psi)(x) = M(x) psi(x) with M [..., 4N, 4N] and psi [..., 4, N]."""
    n = psi.shape[-1]
    flat = psi.reshape(psi.shape[:4] + (4 * n,))
    return np.einsum("...ij,...j->...i", M, flat).reshape(psi.shape)


def expm_hermitian(X):
    """exp(X) of Hermitian matrices [..., n, n] through the eigendecomposition
    X = W diag(lam) W^+ (a library primitive)."""
    lam, W = np.linalg.eigh(X)
    return np.einsum("...ij,...j,...kj->...ik", W, np.exp(lam), np.conj(W))


def clover_diag(U, m0, csw, kind="sw"):
    """Site-diagonal block M(x) of the improved operator and its inverse.

    kind "sw":  M = m + A (Sheikholeslami-Wohlert), inverse by LAPACK.
    kind "exp": M = m exp(A / m) (exponentiated clover; Sec. 2.2 names it
                without a formula, the reading is the one whose first order
                in c_sw is the "sw" term), inverse (1/m) exp(-A / m).
    m = 4 + m0."""
    A = clover(U, csw)
    n4 = A.shape[-1]
    m = 4.0 + m0
    if kind == "sw":
        M = A + m * np.eye(n4)
        return M, np.linalg.inv(M)
    if kind == "exp":
        return m * expm_hermitian(A / m), expm_hermitian(-A / m) / m
    raise ValueError(f"unknown clover kind {kind!r}")


def dirac_clover(U, psi, m0, csw, kind="sw"):
    """D_sw psi = (M - H/2) psi: the Wilson D with its mass term m replaced by M(x)."""
    M, _ = clover_diag(U, m0, csw, kind)
    m = 4.0 + m0
    return dirac(U, psi, m0) - m * psi + apply_site_matrix(M, psi)


def dirac_clover_dagger(U, psi, m0, csw, kind="sw"):
    return apply_gamma5(dirac_clover(U, apply_gamma5(psi), m0, csw, kind))


def dhat_clover(U, psi_e, m0, csw, Mfields=None, kind="sw"):
    """D^ = M_ee - D_eo M_oo^{-1} D_oe on even sites (Schur complement of D_sw)."""
    M, Minv = clover_diag(U, m0, csw, kind) if Mfields is None else Mfields
    psi_e = restrict(psi_e, 0)
    t_o = apply_site_matrix(Minv, hop_block(U, psi_e, 1))
    t_o = restrict(t_o, 1)
    return restrict(apply_site_matrix(M, psi_e), 0) - hop_block(U, t_o, 0)


def dhat_clover_dagger(U, psi_e, m0, csw, Mfields=None, kind="sw"):
    return apply_gamma5(dhat_clover(U, apply_gamma5(psi_e), m0, csw, Mfields, kind))


def cg_clover(U, b_e, m0, csw, tol=1e-10, maxiter=10000, kind="sw"):
    """CG on D^+ D^ for the clover operator."""
    Mf = clover_diag(U, m0, csw, kind)

    def op(v):
        return dhat_clover_dagger(U, dhat_clover(U, v, m0, csw, Mf), m0, csw, Mf)

    return cg(U, b_e, m0, tol=tol, maxiter=maxiter, op=op)


def true_residual_clover(U, b_e, x_e, m0, csw, kind="sw"):
    Mf = clover_diag(U, m0, csw, kind)
    b_e = restrict(_cplx(b_e), 0)
    Ax = dhat_clover_dagger(U, dhat_clover(U, restrict(_cplx(x_e), 0), m0, csw, Mf), m0, csw, Mf)
    return norm(b_e - Ax) / norm(b_e)


# ---------------------------------------------------------------------------
# 16-bit storage: binary16 spinors with a per-site FP32 scale, binary16 links
# (the reduced-precision storage of the mixed-precision solver's inner
# iterations).  The paper does not describe one; this is the definition the
# GPU library's 16-bit format is tested against, bit for bit.
# ---------------------------------------------------------------------------

def quantize_spinor16(psi):
    """Stored form of a spinor field [..., 4, N] (complex): per site, every
    real part and imaginary part is first rounded to FP32; s is the largest of
    their absolute values over the site's 4N components (FP32); each is stored
    as binary16 (round to nearest even) of its FP32 value times the FP32
    reciprocal 1/s.  A site with s = 0 stores zeros.  Both products and the
    reciprocal are single FP32 operations.  Returns (codes, s): codes float16
    [..., 4, N, 2] (re, im), s float32 [...]."""
    f = np.stack([np.real(psi), np.imag(psi)], axis=-1).astype(np.float32)
    s = np.abs(f).reshape(f.shape[:-3] + (-1,)).max(axis=-1)
    safe = np.where(s > 0, s, np.float32(1)).astype(np.float32)
    inv = np.where(s > 0, np.float32(1) / safe, np.float32(0)).astype(np.float32)
    codes = (f * inv[..., None, None, None]).astype(np.float16)
    return codes, s


def dequantize_spinor16(codes, s):
    """The spinor a stored form represents: code * s per real component (an
    11-bit by 24-bit product, exact in FP64)."""
    x = codes.astype(np.float64) * s.astype(np.float64)[..., None, None, None]
    return x[..., 0] + 1j * x[..., 1]


def round_spinor16(psi):
    """psi as stored in the 16-bit format and read back."""
    return dequantize_spinor16(*quantize_spinor16(psi))


def round_links16(U):
    """Links as stored in the 16-bit format and read back: each real entry (re
    and im of complex links) rounded to FP32, then to binary16.  Entries of
    unitary or orthogonal matrices are bounded by 1, so links carry no scale."""
    def r(a):
        return np.asarray(a).astype(np.float32).astype(np.float16).astype(np.float64)

    if np.iscomplexobj(U):
        return r(U.real) + 1j * r(U.imag)
    return r(U)


# ---------------------------------------------------------------------------
# SU(N) and its two-index representations (the paper's Sec. 1: HiRep runs
# SU(N) gauge theories with fermions in the fundamental and higher
# representations).  The representation of a link is the matrix of the
# group action on an orthonormal basis of the representation space; the
# operator's spectrum does not depend on which basis is taken.
# ---------------------------------------------------------------------------

def su_generators(nc):
    """Hermitian traceless generators T_a of su(nc), tr(T_a T_b) = delta_ab / 2:
    the symmetric, antisymmetric and diagonal generalised Gell-Mann matrices, halved."""
    T = []
    for j in range(nc):
        for k in range(j + 1, nc):
            m = np.zeros((nc, nc), np.complex128)
            m[j, k] = m[k, j] = 0.5
            T.append(m)
            m = np.zeros((nc, nc), np.complex128)
            m[j, k] = -0.5j
            m[k, j] = 0.5j
            T.append(m)
    for l in range(1, nc):
        m = np.zeros((nc, nc), np.complex128)
        for j in range(l):
            m[j, j] = 1.0
        m[l, l] = -float(l)
        T.append(m / np.sqrt(2.0 * l * (l + 1)))
    return np.array(T)


def two_index_basis(nc, kind):
    """Orthonormal basis of symmetric ("sym") or antisymmetric ("asym") nc x nc
    matrices (Frobenius inner product), in the order (i, j), i <= j (sym) or
    i < j (asym), row-major."""
    E = []
    for i in range(nc):
        for j in range(i, nc):
            if i == j and kind == "asym":
                continue
            m = np.zeros((nc, nc), np.complex128)
            if i == j:
                m[i, i] = 1.0
            else:
                m[i, j] = 1.0 / np.sqrt(2.0)
                m[j, i] = (1.0 if kind == "sym" else -1.0) / np.sqrt(2.0)
            E.append(m)
    return np.array(E)


def rep_dim(nc, rep):
    return {"fund": nc, "adj": nc * nc - 1, "sym": nc * (nc + 1) // 2, "asym": nc * (nc - 1) // 2}[rep]


def represent(U, rep):
    """Links of the representation rep of SU(nc) from fundamental links U [..., nc, nc]:
      fund : U;
      adj  : R_ab = 2 tr(T_a U T_b U^+), real orthogonal (nc^2 - 1);
      sym  : R_kl = tr(E_k^+ U E_l U^T) over the symmetric basis (nc (nc + 1) / 2);
      asym : the same over the antisymmetric basis (nc (nc - 1) / 2);
    the two-index maps are the action M -> U M U^T of U (x) U on matrices."""
    U = _cplx(U)
    nc = U.shape[-1]
    if rep == "fund":
        return U.copy()
    if rep == "adj":
        T = su_generators(nc)
        Ud = np.conj(np.swapaxes(U, -1, -2))
        R = 2.0 * np.einsum("aij,...jk,bkl,...li->...ab", T, U, T, Ud)
        return R.real.copy()
    E = two_index_basis(nc, rep)
    return np.einsum("kji,...jm,lmn,...in->...kl", np.conj(E), U, E, U)


def represent_backward(U, G, rep):
    """Chain rule of represent(): for L(U) = Re sum conj(G) R(U) (for the real
    adjoint, L = sum G R(U)), return dL/dRe U + i dL/dIm U [..., nc, nc], the
    derivative convention of force().  Evaluated by reverse-mode automatic
    differentiation (torch, CPU, complex128) of the representation map as
    represent() defines it, so it shares no hand-written derivative with the
    GPU library."""
    import torch

    U = _cplx(U)
    nc = U.shape[-1]
    Ut = torch.tensor(U, dtype=torch.complex128, requires_grad=True)
    if rep == "fund":
        R = Ut
    elif rep == "adj":
        T = torch.tensor(su_generators(nc))
        Ud = torch.conj(Ut).transpose(-1, -2)
        R = 2.0 * torch.einsum("aij,...jk,bkl,...li->...ab", T, Ut, T, Ud).real
    else:
        E = torch.tensor(two_index_basis(nc, rep))
        R = torch.einsum("kji,...jm,lmn,...in->...kl", torch.conj(E), Ut, E, Ut)
    Gt = torch.tensor(np.asarray(G))
    L = (Gt.real * R).sum() if rep == "adj" else torch.real(torch.conj(Gt) * R).sum()
    L.backward()
    # torch's gradient of a real function of complex inputs is conj(dL/dz*) * 2 / 2 = dL/dRe + i dL/dIm
    return Ut.grad.detach().numpy().copy()
