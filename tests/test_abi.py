"""The C-ABI library loads and exports every function that include/hrd.h
declares (CPU only: no compute calls), and the pure host-side queries behave
as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hrd.h")
LIB = os.path.join(ROOT, "paper_2411_18511_amd", "libhrd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(hrd_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libhrd.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_api():
    names = declared_functions()
    for must in ("hrd_dirac_apply", "hrd_cg_solve", "hrd_dirac_force", "hrd_dirac_apply_batched",
                 "hrd_cg_solve_batched", "hrd_autotune_batched", "hrd_represent", "hrd_pack_gauge",
                 "hrd_clover_build", "hrd_dirac_apply_clover", "hrd_cg_solve_clover"):
        assert must in names
    assert len(names) >= 28


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_queries(lib):
    class Lat(ctypes.Structure):
        _fields_ = [("dims", ctypes.c_int * 4)]

    lib.hrd_spinor_bytes.restype = ctypes.c_size_t
    lib.hrd_gauge_bytes.restype = ctypes.c_size_t
    lib.hrd_last_error.restype = ctypes.c_char_p
    lib.hrd_version.restype = ctypes.c_char_p
    good = Lat((ctypes.c_int * 4)(8, 8, 8, 8))
    bad = Lat((ctypes.c_int * 4)(8, 8, 8, 7))
    V = 8 ** 4
    assert lib.hrd_spinor_bytes(ctypes.byref(good), 0, 0, 2) == V * 8 * 16
    assert lib.hrd_spinor_bytes(ctypes.byref(good), 1, 1, 1) == V // 2 * 12 * 8
    assert lib.hrd_gauge_bytes(ctypes.byref(good), 0, 0) == V * 4 * 64
    assert lib.hrd_gauge_bytes(ctypes.byref(good), 1, 0) == V * 4 * 72
    assert lib.hrd_spinor_bytes(ctypes.byref(bad), 0, 0, 2) == 0
    assert b"even" in lib.hrd_last_error()
    assert lib.hrd_version().startswith(b"hrd")
    # invalid arguments are rejected before any device work
    lib.hrd_dirac_apply.restype = ctypes.c_int
    assert lib.hrd_dirac_apply(ctypes.byref(bad), 0, 0, None, None, None, ctypes.c_double(0.0), 0, 0, None, None) == 2
    assert lib.hrd_dirac_apply(ctypes.byref(good), 7, 0, None, None, None, ctypes.c_double(0.0), 0, 0, None, None) == 1


def test_clover_queries(lib):
    class Lat(ctypes.Structure):
        _fields_ = [("dims", ctypes.c_int * 4)]

    lib.hrd_clover_bytes.restype = ctypes.c_size_t
    good = Lat((ctypes.c_int * 4)(8, 8, 8, 8))
    V = 8 ** 4
    # 8 N^2 reals per site: N = 2 (FUND, FUND_SU2), 3 (ADJ, ADJ_SU2)
    assert lib.hrd_clover_bytes(ctypes.byref(good), 0, 0) == V * 32 * 8
    assert lib.hrd_clover_bytes(ctypes.byref(good), 2, 1) == V * 32 * 4
    assert lib.hrd_clover_bytes(ctypes.byref(good), 1, 0) == V * 72 * 8
    assert lib.hrd_clover_bytes(ctypes.byref(good), 3, 1) == V * 72 * 4
    assert lib.hrd_clover_bytes(ctypes.byref(good), 9, 0) == 0
    # argument errors before any device work
    lib.hrd_dirac_apply_clover.restype = ctypes.c_int
    assert lib.hrd_dirac_apply_clover(ctypes.byref(good), 0, 0, None, None, None, None, None, 2, 0, None, None) == 1
    assert lib.hrd_dirac_apply_clover(ctypes.byref(good), 0, 0, None, None, None, None, None, 0, 0, None, None) == 1
    lib.hrd_clover_build.restype = ctypes.c_int
    assert lib.hrd_clover_build(ctypes.byref(good), 0, 0, None, ctypes.c_double(1.0), ctypes.c_double(0.0), None,
                                None, None) == 1
    assert lib.hrd_clover_build(ctypes.byref(good), 0, 5, None, ctypes.c_double(1.0), ctypes.c_double(0.0), None,
                                None, None) == 1


@pytest.mark.parametrize("Vh", [1, 8, 63, 64, 65, 128, 360, 720, 1000])
@pytest.mark.parametrize("P,extra", [(1, 0), (2, 0), (4, 0), (8, 0), (3, 4), (1, 2), (4, 8)])
def test_tile_layout_is_a_bijection(Vh, P, extra):
    """The 64-site tile layout documented in include/hrd.h places every
    (plane, site) element and every trailing per-site entry exactly once inside
    the block of Vh sites, without gaps: the block keeps the size of the plane
    layout, Vh (16 P + extra) bytes, for any Vh (ragged last tile included)."""
    import numpy as np

    site = np.arange(Vh)
    b0 = site & ~63
    nb = np.minimum(64, Vh - b0)
    tile = b0 * (16 * P + extra)
    used = np.zeros(Vh * (16 * P + extra), dtype=np.int64)
    for q in range(P):
        off = tile + (q * nb + site - b0) * 16
        assert (off % 16 == 0).all()
        for k in range(16):
            np.add.at(used, off + k, 1)
    if extra:
        off = tile + P * nb * 16 + (site - b0) * extra
        assert (off % extra == 0).all()
        for k in range(extra):
            np.add.at(used, off + k, 1)
    assert (used == 1).all()


def test_library_was_built_from_this_tree(lib):
    """The build compiles the hash of the library sources into libhrd.so, and
    the binding refuses a library whose hash differs from the tree's."""
    from paper_2411_18511_amd import build

    lib.hrd_build_hash.restype = ctypes.c_char_p
    assert lib.hrd_build_hash().decode() == build.source_hash()
    lib.hrd_version.restype = ctypes.c_char_p
    assert build.source_hash().encode() in lib.hrd_version()
