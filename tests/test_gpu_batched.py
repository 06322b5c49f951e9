"""Batched multi-RHS / mixed-volume execution: the persistent batched launches
equal the per-problem launches bitwise (same per-site arithmetic), match the
oracle to the FP32 tolerance, and the batched CG brings every right-hand side
to a true residual <= 1e-10 (oracle recomputation on samples).  The
configuration of 12 right-hand sides on 16^4, 24^3x48 and 32^4 lattices with
both representations mixed is run in full."""
import os
import tempfile

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


def _problem_set(specs, oracle, seed0=200, prec_in="f32"):
    """specs: list of (dims, rep, nrhs, m0).  Returns fields and packed sources."""
    h = hrd()
    out = []
    for i, (dims, rep, nrhs, m0) in enumerate(specs):
        F = Field(dims, rep, seed=seed0 + i)
        psis = [F.spinor(seed0 + 100 * i + k) for k in range(nrhs)]
        if prec_in == "f32":
            src = torch.stack([F.pack(oracle.restrict(p, 0), "f32", "even") for p in psis])
        else:
            src = torch.stack([F.pack(oracle.restrict(p, 0), "f64", "even") for p in psis])
        out.append({"F": F, "dims": dims, "rep": rep, "nrhs": nrhs, "m0": m0, "psis": psis, "src": src,
                    "dst": torch.zeros_like(src)})
    return out


SMALL = [((4, 4, 4, 4), "fund", 3, -0.2), ((6, 4, 6, 10), "adj", 5, -0.5), ((8, 8, 8, 8), "fund", 2, -0.3),
         ((4, 24, 48, 48), "fund", 2, -0.3)]


@pytest.mark.parametrize("parity", ["eo", "hop_eo", "hop_oe"])
@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("tune", [None, {"sites_per_tile": 64, "rhs_per_tile": 3, "block_threads": 64,
                                         "blocks_per_cu": 2},
                                  {"sites_per_tile": 256, "rhs_per_tile": 6, "block_threads": 256,
                                   "blocks_per_cu": 8},
                                  {"sites_per_tile": 128, "rhs_per_tile": 12, "block_threads": 128,
                                   "blocks_per_cu": 4, "slab_width": 2},
                                  {"sites_per_tile": 64, "rhs_per_tile": 2, "block_threads": 64,
                                   "blocks_per_cu": 4, "slab_width": 1}])
def test_batched_equals_single(oracle, parity, dagger, tune):
    h = hrd()
    ps = _problem_set(SMALL, oracle)
    if parity == "hop_eo":  # sources live on odd sites
        for p in ps:
            p["src"] = torch.stack([p["F"].pack(oracle.restrict(q, 1), "f32", "odd") for q in p["psis"]])
    probs = h.make_problems([{"dims": p["dims"], "rep": p["rep"], "nrhs": p["nrhs"], "m0": p["m0"],
                              "U32": p["F"].U32, "src": p["src"], "dst": p["dst"]} for p in ps])
    h.dirac_apply_batched(probs, parity, dagger=dagger, tune=tune)
    torch.cuda.synchronize()
    for p in ps:
        for k in range(p["nrhs"]):
            single = h.dirac_apply(p["F"].U32, p["src"][k], p["m0"], p["rep"], parity, p["dims"], prec="f32",
                                   dagger=dagger)
            assert torch.equal(single, p["dst"][k]), (p["dims"], p["rep"], k)
    # and the FP32 tolerance against the oracle for one right-hand side per problem
    out_sites = {"eo": "even", "hop_eo": "even", "hop_oe": "odd"}[parity]
    for p in ps:
        got = p["F"].unpack(p["dst"][0], "f32", out_sites)
        q = p["psis"][0]
        U = p["F"].U_orc
        if parity == "eo":
            e = oracle.restrict(q, 0)
            want = oracle.dhat_dagger(U, e, p["m0"]) if dagger else oracle.dhat(U, e, p["m0"])
        else:
            tgt = 0 if parity == "hop_eo" else 1
            f = oracle.hop_block_dagger if dagger else oracle.hop_block
            want = f(U, q, tgt)
        assert rel_err(got, want) <= 1e-6


def test_batched_errors():
    h = hrd()
    with pytest.raises(h.HrdError):
        h.dirac_apply_batched(h.make_problems([]), "eo")
    F = Field((4, 4, 4, 4), "fund", seed=1)
    src = torch.zeros(h.spinor_bytes((4, 4, 4, 4), "fund", "f32", 1), dtype=torch.uint8, device="cuda")
    probs = h.make_problems([{"dims": (4, 4, 4, 4), "rep": "fund", "nrhs": 1, "m0": -0.2, "U32": F.U32,
                              "src": src, "dst": src}])
    with pytest.raises(h.HrdError) as e:
        h.dirac_apply_batched(probs, "eo")
    assert e.value.status == h.EALIAS
    dst = torch.zeros_like(src)
    probs = h.make_problems([{"dims": (4, 4, 4, 4), "rep": "fund", "nrhs": 1, "m0": -0.2, "U32": F.U32,
                              "src": src, "dst": dst}])
    with pytest.raises(h.HrdError) as e:
        h.dirac_apply_batched(probs, "eo", tune={"sites_per_tile": 96, "rhs_per_tile": 1, "block_threads": 96,
                                                 "blocks_per_cu": 2})
    assert e.value.status == h.EINVAL


CONFIG4 = [((16, 16, 16, 16), "fund", 12, -0.3), ((48, 24, 24, 24), "fund", 12, -0.3),
           ((32, 32, 32, 32), "fund", 12, -0.3), ((16, 16, 16, 16), "adj", 12, -0.5),
           ((48, 24, 24, 24), "adj", 12, -0.5), ((32, 32, 32, 32), "adj", 12, -0.5)]


def test_batched_cg_config4(oracle):
    """12 right-hand sides on each of 16^4, 24^3x48, 32^4, fund and adjoint: one
    batched mixed-precision CG; oracle true residual on two right-hand sides per
    problem, the library's FP64 residual on all of them."""
    h = hrd()
    ps = _problem_set(CONFIG4, oracle, seed0=400, prec_in="f64")
    probs = h.make_problems([{"dims": p["dims"], "rep": p["rep"], "nrhs": p["nrhs"], "m0": p["m0"],
                              "U32": p["F"].U32, "U64": p["F"].U64, "src": p["src"], "dst": p["dst"]}
                             for p in ps])
    infos, status = h.cg_solve_batched(probs, 1e-10)
    assert status == "HRD_OK"
    assert len(infos) == 72
    assert max(i["true_rel_residual"] for i in infos) <= 1e-10
    print("iterations", [i["iters"] for i in infos])
    r = 0
    for p in ps:
        for k in (0, p["nrhs"] - 1):
            x = p["F"].unpack(p["dst"][k], "f64", "even")
            b = oracle.restrict(p["psis"][k], 0)
            res = oracle.true_residual(p["F"].U_orc, b, x, p["m0"])
            assert res <= 1e-10, (p["dims"], p["rep"], k, res)


def test_batched_cg_matches_single_solves(oracle):
    h = hrd()
    specs = [((4, 4, 4, 4), "fund", 3, -0.2), ((6, 4, 6, 10), "adj", 2, -0.5)]
    ps = _problem_set(specs, oracle, seed0=500, prec_in="f64")
    probs = h.make_problems([{"dims": p["dims"], "rep": p["rep"], "nrhs": p["nrhs"], "m0": p["m0"],
                              "U32": p["F"].U32, "U64": p["F"].U64, "src": p["src"], "dst": p["dst"]}
                             for p in ps])
    infos, status = h.cg_solve_batched(probs, 1e-10)
    assert status == "HRD_OK"
    r = 0
    for p in ps:
        for k in range(p["nrhs"]):
            xs, inf = h.cg_solve(p["F"].U64, p["src"][k], p["m0"], 1e-10, p["dims"], p["rep"], mode="mixed",
                                 U32=p["F"].U32)
            xb = p["F"].unpack(p["dst"][k], "f64", "even")
            assert rel_err(xb, p["F"].unpack(xs, "f64", "even")) < 1e-7
            assert infos[r]["true_rel_residual"] <= 1e-10
            r += 1
    # maxiter too small: ENOCONV with every info filled
    for p in ps:
        p["dst"].zero_()
    infos, status = h.cg_solve_batched(probs, 1e-10, maxiter=3, allow_noconv=True)
    assert status == "HRD_ENOCONV" and all(i["iters"] == 3 for i in infos)


def test_autotune_and_cache(oracle):
    h = hrd()
    ps = _problem_set([((8, 8, 8, 8), "fund", 4, -0.2), ((6, 4, 6, 10), "adj", 3, -0.5)], oracle, seed0=600)
    probs = h.make_problems([{"dims": p["dims"], "rep": p["rep"], "nrhs": p["nrhs"], "m0": p["m0"],
                              "U32": p["F"].U32, "src": p["src"], "dst": p["dst"]} for p in ps])
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.jsonl")
        best = h.autotune_batched(probs, cache_path=path)
        assert best["sites_per_tile"] in (64, 128, 256) and best["rhs_per_tile"] in (1, 2, 4, 6, 12)
        assert os.path.exists(path) and "gfx" in open(path).read()
        again = h.autotune_batched(probs, cache_path=path)
        assert again == best
        # the tuned shape computes the same result
        h.dirac_apply_batched(probs, "eo", tune=best)
        torch.cuda.synchronize()
        for p in ps:
            single = h.dirac_apply(p["F"].U32, p["src"][0], p["m0"], p["rep"], "eo", p["dims"], prec="f32")
            assert torch.equal(single, p["dst"][0])
