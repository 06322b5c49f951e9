"""Helpers for the GPU parity tests: move seeded numpy fields to the GPU in the
natural layout, run the library through its binding, bring results back.

The oracle and the library both consume the arrays produced by
``paper_2411_18511_amd.inputs``; nothing here computes any part of the method.
"""
import numpy as np
import pytest
import torch

from paper_2411_18511_amd import inputs

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def hrd():
    from paper_2411_18511_amd import hrd as _h

    return _h


def to_dev_spinor(psi):
    """numpy [T, L1, L2, L3, 4, N] -> cuda complex128 [V, 4, N]."""
    V = int(np.prod(psi.shape[:4]))
    return torch.from_numpy(np.ascontiguousarray(psi.reshape(V, 4, psi.shape[-1]))).cuda()


def from_dev_spinor(t, dims):
    n = t.shape[-1]
    return t.cpu().numpy().reshape(tuple(dims) + (4, n))


def to_dev_gauge(U):
    """numpy [4, T, L1, L2, L3, N, N] -> cuda [4, V, N, N] (complex128 or float64)."""
    V = int(np.prod(U.shape[1:5]))
    return torch.from_numpy(np.ascontiguousarray(U.reshape(4, V, U.shape[-2], U.shape[-1]))).cuda()


def from_dev_gauge(t, dims):
    return t.cpu().numpy().reshape((4,) + tuple(dims) + tuple(t.shape[-2:]))


def tile_index(Vh, site, q, P):
    """Position, in 16-byte elements, of plane q of `site` in a block of Vh
    sites with P planes stored in 64-site tiles (the layout include/hrd.h
    documents): tile t = site // 64 holds plane 0 of its nb sites, then plane
    1, ...; nb = 64 except in the last tile."""
    site = np.asarray(site)
    b0 = site & ~63
    nb = np.minimum(64, Vh - b0)
    return b0 * P + q * nb + (site - b0)


def rel_err(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def site_rel_err(a, b):
    """Largest per-site relative error max_x ||a(x) - b(x)|| / ||b(x)|| over the
    sites where b(x) is nonzero (fields [T, L1, L2, L3, 4, N] or [..., N, N]);
    sites where b(x) = 0 must have a(x) = 0 exactly."""
    a = np.asarray(a).reshape(int(np.prod(a.shape[:4])), -1)
    b = np.asarray(b).reshape(a.shape)
    nb = np.linalg.norm(b, axis=1)
    nd = np.linalg.norm(a - b, axis=1)
    zero = nb == 0
    assert np.all(nd[zero] == 0), "output nonzero where the reference is zero"
    return float((nd[~zero] / nb[~zero]).max()) if (~zero).any() else 0.0


class Field:
    """A seeded problem: fundamental links, optional adjoint links, packed on the GPU."""

    def __init__(self, dims, rep, seed, kind="haar"):
        import oracle as O

        h = hrd()
        self.dims = tuple(dims)
        self.rep = rep
        self.n = 2 if rep in ("fund", "fund_su2") else 3
        self.Uf = inputs.gauge_field(dims, seed, kind=kind)
        self.Uf_dev = to_dev_gauge(self.Uf)
        Uf64 = h.pack_gauge(self.Uf_dev, dims, "fund", "f64")
        if self.n == 2:
            self.U_orc = self.Uf
        else:
            self.U_orc = O.represent_adjoint(self.Uf).astype(np.complex128)
        if rep == "fund":
            self.U64 = Uf64
        elif rep == "adj":
            self.U64 = h.represent(Uf64, dims, "f64")
        else:  # links stored as the first row of the fundamental matrix
            self.U64 = h.pack_gauge(self.Uf_dev, dims, rep, "f64")
        self.Uf64 = Uf64
        self.U32 = h.convert_gauge(self.U64, dims, rep)

    def spinor(self, seed):
        return inputs.gaussian_spinor(self.dims, self.n, seed)

    def pack(self, psi, prec="f64", sites="all"):
        return hrd().pack_spinor(to_dev_spinor(psi), self.dims, self.rep, prec, sites)

    def unpack(self, packed, prec="f64", sites="all"):
        out = hrd().unpack_spinor(packed, self.dims, self.rep, prec, sites)
        return from_dev_spinor(out, self.dims)


class FieldSUN:
    """A seeded SU(nc) problem in representation `rep` ('fund', 'adj', 'sym',
    'asym'): fundamental links packed on the GPU (format CPLXnc), the
    representation built by the library, FP32 and F16 copies; the oracle gets
    the representation computed by its own map."""

    def __init__(self, dims, nc, rep, seed, kind="haar"):
        import oracle as O

        h = hrd()
        self.dims = tuple(dims)
        self.nc = nc
        self.fmt = h.sun_rep_format(nc, rep)
        self.rep = self.fmt
        self.n = h.ncolour(self.fmt)
        self.Uf = inputs.gauge_field_sun(dims, seed, nc, kind=kind)
        Uf64 = h.pack_gauge(to_dev_gauge(self.Uf), dims, "cplx3" if nc == 3 else "cplx4", "f64")
        self.U64 = h.represent_sun(Uf64, dims, nc, rep)
        self.U32 = h.convert_gauge_prec(self.U64, dims, self.fmt, "f32")
        self.U16 = h.convert_gauge_prec(self.U64, dims, self.fmt, "f16")
        self.U_orc = O.represent(self.Uf, rep).astype(np.complex128)

    def spinor(self, seed):
        return inputs.gaussian_spinor(self.dims, self.n, seed)

    def pack(self, psi, prec="f64", sites="all"):
        h = hrd()
        if prec == "f16":
            np_ = 2 if sites == "all" else 1
            return h.convert_spinor_prec(h.pack_spinor(to_dev_spinor(psi), self.dims, self.fmt, "f64", sites),
                                         self.dims, self.fmt, np_, "f64", "f16")
        return h.pack_spinor(to_dev_spinor(psi), self.dims, self.fmt, prec, sites)

    def unpack(self, packed, prec="f64", sites="all"):
        h = hrd()
        if prec == "f16":
            np_ = 2 if sites == "all" else 1
            packed = h.convert_spinor_prec(packed, self.dims, self.fmt, np_, "f16", "f64")
            prec = "f64"
        return from_dev_spinor(h.unpack_spinor(packed, self.dims, self.fmt, prec, sites), self.dims)
