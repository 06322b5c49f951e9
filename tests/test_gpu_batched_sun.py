"""Batched launches for the dense SU(N > 2) link formats (Sec. 1: SU(N) with
fermions in higher representations): a batch of problems sharing one dense
format (mixed volumes, and for CPLX3 two representations, SU(3) fundamental
and antisymmetric) equals the per-problem launches bit for bit, matches the
oracle to the FP32 tolerance, and the batched CG brings every right-hand side
to a true residual <= 1e-10 (oracle recomputation on samples)."""
import numpy as np
import pytest
import torch

from gpu_util import FieldSUN, requires_gpu, rel_err, hrd

pytestmark = [pytest.mark.gpu, requires_gpu]

# format -> list of (nc, rep, dims, nrhs, m0); every problem of a batch shares the format
BATCHES = {
    "cplx3": [(3, "fund", (4, 4, 4, 4), 3, -0.3), (3, "asym", (6, 4, 6, 10), 2, -0.2)],
    "cplx4": [(4, "fund", (4, 4, 4, 4), 2, -0.3), (4, "fund", (4, 2, 2, 6), 3, -0.1)],
    "cplx6": [(3, "sym", (4, 4, 4, 4), 2, -0.3), (4, "asym", (4, 2, 4, 6), 2, -0.2)],
    "real8": [(3, "adj", (4, 4, 4, 4), 2, -0.3), (3, "adj", (6, 4, 6, 10), 2, -0.4)],
    "cplx10": [(4, "sym", (4, 2, 2, 6), 2, -0.3)],
    "real15": [(4, "adj", (4, 2, 2, 6), 2, -0.3)],
}


@pytest.fixture(scope="module")
def oracle():
    import oracle as O

    O._load()
    return O


def _batch(oracle, specs, seed0, prec):
    out = []
    for i, (nc, rep, dims, nrhs, m0) in enumerate(specs):
        F = FieldSUN(dims, nc, rep, seed=seed0 + i)
        psis = [F.spinor(seed0 + 50 * i + k) for k in range(nrhs)]
        src = torch.stack([F.pack(oracle.restrict(p, 0), prec, "even") for p in psis])
        out.append({"F": F, "dims": dims, "nrhs": nrhs, "m0": m0, "psis": psis, "src": src,
                    "dst": torch.zeros_like(src)})
    return out


def _problems(h, ps):
    return h.make_problems([{"dims": p["dims"], "rep": p["F"].fmt, "nrhs": p["nrhs"], "m0": p["m0"],
                             "U32": p["F"].U32, "U64": p["F"].U64, "src": p["src"], "dst": p["dst"]} for p in ps])


@pytest.mark.parametrize("fmt", list(BATCHES))
@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("tune", [None, {"sites_per_tile": 64, "rhs_per_tile": 2, "block_threads": 64,
                                         "blocks_per_cu": 2, "slab_width": 1}])
def test_dense_batched_equals_single(oracle, fmt, dagger, tune):
    h = hrd()
    ps = _batch(oracle, BATCHES[fmt], 700, "f32")
    h.dirac_apply_batched(_problems(h, ps), "eo", dagger=dagger, tune=tune)
    torch.cuda.synchronize()
    for p in ps:
        F = p["F"]
        for k in range(p["nrhs"]):
            single = h.dirac_apply(F.U32, p["src"][k], p["m0"], F.fmt, "eo", p["dims"], prec="f32", dagger=dagger)
            assert torch.equal(single, p["dst"][k]), (fmt, p["dims"], k)
        e = oracle.restrict(p["psis"][0], 0)
        want = (oracle.dhat_dagger if dagger else oracle.dhat)(F.U_orc, e, p["m0"])
        assert rel_err(F.unpack(p["dst"][0], "f32", "even"), want) <= 1e-6


@pytest.mark.parametrize("fmt", ["cplx3", "cplx6", "real8", "cplx10"])
def test_dense_batched_cg(oracle, fmt):
    h = hrd()
    ps = _batch(oracle, BATCHES[fmt], 800, "f64")
    infos, status = h.cg_solve_batched(_problems(h, ps), 1e-10)
    assert status == "HRD_OK"
    assert max(i["true_rel_residual"] for i in infos) <= 1e-10
    for p in ps:
        F = p["F"]
        for k in (0, p["nrhs"] - 1):
            x = F.unpack(p["dst"][k], "f64", "even")
            b = oracle.restrict(p["psis"][k], 0)
            assert oracle.true_residual(F.U_orc, b, x, p["m0"]) <= 1e-10, (fmt, p["dims"], k)


def test_dense_batched_format_mix_rejected():
    h = hrd()
    a = FieldSUN((4, 4, 4, 4), 3, "fund", seed=901)
    b = FieldSUN((4, 4, 4, 4), 3, "sym", seed=902)
    specs = []
    for F in (a, b):
        src = torch.zeros((1, h.spinor_bytes(F.dims, F.fmt, "f32", 1)), dtype=torch.uint8, device="cuda")
        specs.append({"dims": F.dims, "rep": F.fmt, "nrhs": 1, "m0": -0.3, "U32": F.U32, "src": src,
                      "dst": torch.zeros_like(src)})
    with pytest.raises(h.HrdError) as e:
        h.dirac_apply_batched(h.make_problems(specs), "eo")
    assert e.value.status == h.EINVAL
