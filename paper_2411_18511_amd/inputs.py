"""Seeded synthetic inputs: SU(2) and SU(N) gauge fields, Gaussian spinor fields.

This module holds no part of the Dirac operator, the solver or the force; it
only draws random fields, in the natural layout

* gauge links  ``U[mu, t, x1, x2, x3, i, j]`` complex128 (fundamental SU(2)),
* spinors      ``psi[t, x1, x2, x3, spin, colour]`` complex128,

with numpy's PCG64 generator.  Both the GPU library's tests and the CPU
oracle consume the same arrays.

The paper timed its operator on gauge fields it does not describe (Sec. 3,
Table 1); bandwidth does not depend on field content, so these stand in:

* Haar-random links: a = g / |g| with g ~ N(0, 1)^4 and
  U = a0 + i (a1 s1 + a2 s2 + a3 s3)  (uniform on SU(2) = S^3).
* "Heat-bath-like" links: a = (1, eps g1, eps g2, eps g3) / norm, i.e. Haar
  directions pulled toward the identity.  For independent links the mean
  plaquette is E[a0]^4, so eps is chosen by bisection to make E[a0]^4 equal
  the requested plaquette (0.6 by default).
* SU(N) links (N >= 2): Haar-random unitary matrices from the QR
  factorisation of a complex Gaussian matrix with the phases of R's diagonal
  divided out (Mezzadri's method), then divided by an N-th root of the
  determinant; "smeared" SU(N) links are exp(i eps H) with H a Gaussian
  traceless Hermitian matrix (near the identity); "product" SU(N) links are
  products of Haar SU(2) elements embedded in every 2x2 block (fast to draw
  on large lattices).
* Spinors: real and imaginary parts i.i.d. N(0, 1/2).
"""
import numpy as np


def rng_for(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _su2_from_quaternion(a):
    """U = a0 + i a.s for unit 4-vectors a (last axis); returns [..., 2, 2]."""
    a0, a1, a2, a3 = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    U = np.empty(a.shape[:-1] + (2, 2), np.complex128)
    U[..., 0, 0] = a0 + 1j * a3
    U[..., 0, 1] = a2 + 1j * a1
    U[..., 1, 0] = -a2 + 1j * a1
    U[..., 1, 1] = a0 - 1j * a3
    return U


def haar_su2(rng, shape):
    g = rng.standard_normal(tuple(shape) + (4,))
    g /= np.linalg.norm(g, axis=-1, keepdims=True)
    return _su2_from_quaternion(g)


def _mean_a0(eps):
    """E[1 / sqrt(1 + eps^2 r^2)] for r ~ chi(3), by quadrature on a fine grid."""
    r = np.linspace(0.0, 12.0, 200001)
    w = np.sqrt(2.0 / np.pi) * r * r * np.exp(-0.5 * r * r)
    f = w / np.sqrt(1.0 + (eps * r) ** 2)
    return float(np.trapezoid(f, r) / np.trapezoid(w, r))


def smearing_for_plaquette(target=0.6):
    """eps such that E[a0]^4 == target for the heat-bath-like generator."""
    lo, hi = 0.0, 50.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if _mean_a0(mid) ** 4 > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def smeared_su2(rng, shape, eps):
    g = rng.standard_normal(tuple(shape) + (3,))
    a = np.concatenate([np.ones(tuple(shape) + (1,)), eps * g], axis=-1)
    a /= np.linalg.norm(a, axis=-1, keepdims=True)
    return _su2_from_quaternion(a)


def gauge_field(dims, seed, kind="haar", plaquette=0.6):
    """Fundamental SU(2) gauge field [4, T, L1, L2, L3, 2, 2] (complex128)."""
    rng = rng_for(seed)
    shape = (4,) + tuple(int(d) for d in dims)
    if kind == "haar":
        return haar_su2(rng, shape)
    if kind == "smeared":
        return smeared_su2(rng, shape, smearing_for_plaquette(plaquette))
    if kind == "unit":
        U = np.zeros(shape + (2, 2), np.complex128)
        U[..., 0, 0] = 1
        U[..., 1, 1] = 1
        return U
    raise ValueError(f"unknown gauge kind {kind!r}")


def haar_sun(rng, shape, nc):
    """Haar-random SU(nc) matrices [..., nc, nc]."""
    shape = tuple(shape)
    z = (rng.standard_normal(shape + (nc, nc)) + 1j * rng.standard_normal(shape + (nc, nc))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / nc))[..., None, None]


def smeared_sun(rng, shape, nc, eps=0.35):
    """SU(nc) matrices exp(i eps H), H Gaussian, Hermitian and traceless."""
    shape = tuple(shape)
    z = rng.standard_normal(shape + (nc, nc)) + 1j * rng.standard_normal(shape + (nc, nc))
    h = (z + np.conj(np.swapaxes(z, -1, -2))) / 2
    h = h - np.trace(h, axis1=-2, axis2=-1)[..., None, None] * np.eye(nc) / nc
    w, v = np.linalg.eigh(h)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * eps * w), np.conj(v))


def subgroup_product_sun(rng, shape, nc):
    """SU(nc) matrices as products of Haar SU(2) elements embedded in every
    (i, j) 2x2 block, i < j (cheap to draw for large lattices; not Haar on
    SU(nc), but spread over the group)."""
    shape = tuple(shape)
    U = np.broadcast_to(np.eye(nc, dtype=np.complex128), shape + (nc, nc)).copy()
    for i in range(nc):
        for j in range(i + 1, nc):
            s2 = haar_su2(rng, shape)
            # right-multiply by the embedded block: columns i and j of U mix
            ci, cj = U[..., :, i].copy(), U[..., :, j].copy()
            U[..., :, i] = ci * s2[..., 0, 0, None] + cj * s2[..., 1, 0, None]
            U[..., :, j] = ci * s2[..., 0, 1, None] + cj * s2[..., 1, 1, None]
    return U


def gauge_field_sun(dims, seed, nc, kind="haar"):
    """Fundamental SU(nc) gauge field [4, T, L1, L2, L3, nc, nc] (complex128)."""
    if nc == 2:
        return gauge_field(dims, seed, kind=kind)
    rng = rng_for(seed)
    shape = (4,) + tuple(int(d) for d in dims)
    if kind == "haar":
        return haar_sun(rng, shape, nc)
    if kind == "smeared":
        return smeared_sun(rng, shape, nc)
    if kind == "product":
        return subgroup_product_sun(rng, shape, nc)
    if kind == "unit":
        return np.broadcast_to(np.eye(nc, dtype=np.complex128), shape + (nc, nc)).copy()
    raise ValueError(f"unknown gauge kind {kind!r}")


def gaussian_spinor(dims, ncolour, seed, nrhs=None):
    """Gaussian spinor field [T, L1, L2, L3, 4, N] (or [nrhs, ...]), complex128."""
    rng = rng_for(seed)
    shape = tuple(int(d) for d in dims) + (4, int(ncolour))
    if nrhs is not None:
        shape = (int(nrhs),) + shape
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * np.sqrt(0.5)


def gauge_transform(rng, dims, nc=2):
    """Random site-local SU(nc) matrices g(x), shape [T, L1, L2, L3, nc, nc]."""
    if nc == 2:
        return haar_su2(rng, tuple(int(d) for d in dims))
    return haar_sun(rng, tuple(int(d) for d in dims), nc)
