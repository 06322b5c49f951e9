"""Benchmark of the single-GPU hot path on the 48^4 SU(2) workload.

Workload (the paper's per-GPU weak-scaling share, Table 1): a 48^4 lattice,
SU(2) fundamental fermions, heat-bath-like links (mean plaquette 0.6),
m0 = -0.3, Gaussian complex128 source; synthetic seeded inputs, resident in
HBM before timing starts.

One step = one pass over every stage of the hot path:
  1. gauge preparation: pack the natural links, FP32 copy;
  2. the Dslash: R applications of the FP64 hopping block D_eo and of the FP32
     one, timed with HIP events on the library's stream; plain D and the
     even/odd D^ (and dagger) in FP64 and FP32;
  3. CG on D^+D^ to true residual 1e-10 in FP64 and in mixed precision;
  4. the fermion-action force from the mixed solution;
  5. a batched 12-right-hand-side FP32 D^ in persistent launches (when the
     library provides it).

Prints one JSON line.  `value` is the FP64 Dslash (hopping block) bandwidth
on algorithmic bytes: each link, each source spinor and each output spinor
counted once per application.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "Dslash GB/s & %HBM peak at 48^4 SU(2); mixed vs FP64 CG time to 1e-10"

LINK_BYTES = {("fund", "f64"): 64, ("fund", "f32"): 32, ("adj", "f64"): 72, ("adj", "f32"): 36}
SPINOR_BYTES = {("fund", "f64"): 128, ("fund", "f32"): 64, ("adj", "f64"): 192, ("adj", "f32"): 96}


def hop_alg_bytes(V, rep, prec):
    """Algorithmic bytes of one hopping-block application (V/2 target sites):
    8 links, the source spinor and the output spinor per target site."""
    L, S = LINK_BYTES[(rep, prec)], SPINOR_BYTES[(rep, prec)]
    return (V // 2) * (8 * L + 2 * S)


def full_alg_bytes(V, rep, prec):
    """Algorithmic bytes of the plain D on all V sites: each link once, psi and out once."""
    L, S = LINK_BYTES[(rep, prec)], SPINOR_BYTES[(rep, prec)]
    return V * (4 * L + 2 * S)


def dhat_alg_bytes(V, rep, prec):
    """D^ = two hops plus the m*psi read of the second: V (8L + 2.5 S)."""
    L, S = LINK_BYTES[(rep, prec)], SPINOR_BYTES[(rep, prec)]
    return V * (8 * L) + (V // 2) * 5 * S


def cpu_oracle_sample(U_nat, psi_nat, V, budget_s=10.0):
    """Time the oracle's hopping term (target parity even) on the full lattice."""
    import oracle as O

    O._load()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = 0
    t0 = time.perf_counter()
    while True:
        O.hopping(U_nat, psi_nat, 1)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            break
    gbs = n * hop_alg_bytes(V, "fund", "f64") / dt / 1e9
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} FP64 hopping-block applications (even targets) of the oracle on the full "
                      f"{'x'.join(map(str, U_nat.shape[1:5]))} fundamental lattice in {dt:.1f} s, "
                      f"same algorithmic byte count per application as the GPU figure"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--reps", type=int, default=50, help="Dslash applications timed per step")
    ap.add_argument("--dims", type=str, default="48,48,48,48")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the lattice is not sharded "
                                   "across GPUs (see the design notes on sharding)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import __graft_entry__  # noqa: F401  (puts the repo root on sys.path)
    from paper_2411_18511_amd import hrd, inputs

    dims = tuple(int(x) for x in args.dims.split(","))
    V = int(np.prod(dims))
    m0, tol = -0.3, 1e-10
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    print(f"[bench] generating {dims} inputs", file=sys.stderr, flush=True)
    U_np = inputs.gauge_field(dims, 3, kind="smeared")
    psi_np = inputs.gaussian_spinor(dims, 2, 4)
    U_nat = torch.from_numpy(U_np.reshape(4, V, 2, 2)).to(dev)
    psi_nat = torch.from_numpy(psi_np.reshape(V, 4, 2)).to(dev)
    torch.cuda.synchronize()

    nrhs_batched = 12
    batched_ok = hrd.has_batched() and not args.no_batched
    if batched_ok:
        rhs_np = [inputs.gaussian_spinor(dims, 2, 100 + k) for k in range(nrhs_batched)]
        rhs_nat = [torch.from_numpy(r.reshape(V, 4, 2)).to(dev) for r in rhs_np]
        del rhs_np

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    results = {}

    def step():
        r = {}
        # 1. gauge preparation
        U64 = hrd.pack_gauge(U_nat, dims, "fund", "f64")
        U32 = hrd.convert_gauge(U64, dims, "fund")
        src_all = hrd.pack_spinor(psi_nat, dims, "fund", "f64", "all")
        src_e = hrd.pack_spinor(psi_nat, dims, "fund", "f64", "even")
        src_o = hrd.pack_spinor(psi_nat, dims, "fund", "f64", "odd")
        src_o32 = hrd.convert_spinor(src_o, dims, "fund", 1, True)
        src_e32 = hrd.convert_spinor(src_e, dims, "fund", 1, True)
        out_e = torch.empty_like(src_e)
        out_e32 = torch.empty_like(src_e32)
        out_all = torch.empty_like(src_all)

        # 2. Dslash phases, HIP events on the library's stream
        def timed(fn, reps):
            a, b = ev(), ev()
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            b.synchronize()
            return a.elapsed_time(b) / reps  # ms per application

        R = args.reps
        hop64 = hrd.DiracOp(U64, dims, "fund", "f64", m0, "hop_eo")
        hop32 = hrd.DiracOp(U32, dims, "fund", "f32", m0, "hop_eo")
        full64 = hrd.DiracOp(U64, dims, "fund", "f64", m0, "full")
        dhat64 = hrd.DiracOp(U64, dims, "fund", "f64", m0, "eo")
        dhatd64 = hrd.DiracOp(U64, dims, "fund", "f64", m0, "eo", dagger=True)
        dhat32 = hrd.DiracOp(U32, dims, "fund", "f32", m0, "eo")
        r["hop_f64_ms"] = timed(lambda: hop64(src_o, out_e), R)
        r["hop_f32_ms"] = timed(lambda: hop32(src_o32, out_e32), R)
        r["full_f64_ms"] = timed(lambda: full64(src_all, out_all), R // 2)
        r["dhat_f64_ms"] = timed(lambda: dhat64(src_e, out_e), R // 2)
        r["dhat_dag_f64_ms"] = timed(lambda: dhatd64(src_e, out_e), R // 2)
        r["dhat_f32_ms"] = timed(lambda: dhat32(src_e32, out_e32), R // 2)

        # 3. CG solves (each synchronises internally); events bracket them
        a, b = ev(), ev()
        a.record()
        x64, i64 = hrd.cg_solve(U64, src_e, m0, tol, dims, "fund", mode="f64")
        b.record()
        b.synchronize()
        r["cg_f64_ms"] = a.elapsed_time(b)
        r["cg_f64"] = i64
        a, b = ev(), ev()
        a.record()
        xm, im = hrd.cg_solve(U64, src_e, m0, tol, dims, "fund", mode="mixed", U32=U32)
        b.record()
        b.synchronize()
        r["cg_mixed_ms"] = a.elapsed_time(b)
        r["cg_mixed"] = im
        # x_mixed vs x_f64: both solved to 1e-10
        n64 = hrd.blas_norm2(x64, dims, "fund", "f64", 1)
        d = xm.clone()
        hrd.blas_axpy(-1.0, x64, d, dims, "fund", "f64", 1)
        r["mixed_vs_f64_rel"] = float(np.sqrt(hrd.blas_norm2(d, dims, "fund", "f64", 1) / n64))

        # 4. fermion force from the mixed solution
        a, b = ev(), ev()
        a.record()
        hrd.action_force(U64, xm, m0, dims, "fund")
        b.record()
        b.synchronize()
        r["action_force_ms"] = a.elapsed_time(b)

        # 5. batched multi-RHS D^ (FP32)
        if batched_ok:
            srcs = torch.stack([hrd.convert_spinor(hrd.pack_spinor(t, dims, "fund", "f64", "even"), dims, "fund",
                                                   1, True) for t in rhs_nat])
            dsts = torch.empty_like(srcs)
            probs = hrd.make_problems([{"dims": dims, "rep": "fund", "nrhs": nrhs_batched, "m0": m0, "U32": U32,
                                        "src": srcs, "dst": dsts}])
            wb = torch.empty(max(hrd.batched_workspace_bytes(probs, "eo"), 1), dtype=torch.uint8, device=dev)
            r["batched_dhat_ms"] = timed(lambda: hrd.dirac_apply_batched(probs, "eo", work=wb), 5)
        return r

    for w in range(args.warmup):
        print(f"[bench] warmup {w}", file=sys.stderr, flush=True)
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = []
    for s in range(args.steps):
        per.append(step())
        print(f"[bench] step {s} done: hop f64 {per[-1]['hop_f64_ms']:.3f} ms, cg f64 {per[-1]['cg_f64_ms']:.1f} ms,"
              f" cg mixed {per[-1]['cg_mixed_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    def avg(k):
        return float(np.mean([p[k] for p in per]))

    hop_ms = avg("hop_f64_ms")
    hop_gbs = hop_alg_bytes(V, "fund", "f64") / (hop_ms * 1e-3) / 1e9
    dslash = {
        "hop_f64": {"ms": hop_ms, "alg_GBs": hop_gbs, "site_updates_per_s": (V // 2) / (hop_ms * 1e-3)},
    }
    for key, fn, prec in [("hop_f32", hop_alg_bytes, "f32"), ("full_f64", full_alg_bytes, "f64"),
                          ("dhat_f64", dhat_alg_bytes, "f64"), ("dhat_dag_f64", dhat_alg_bytes, "f64"),
                          ("dhat_f32", dhat_alg_bytes, "f32")]:
        ms = avg(key + "_ms")
        sites = V // 2 if key.startswith("hop") else V
        dslash[key] = {"ms": ms, "alg_GBs": fn(V, "fund", prec) / (ms * 1e-3) / 1e9,
                       "site_updates_per_s": sites / (ms * 1e-3)}
    for v in dslash.values():
        v["pct_hbm_peak"] = 100.0 * v["alg_GBs"] / HBM_PEAK_GBS
    cg = {
        "f64": {"ms": avg("cg_f64_ms"), **per[-1]["cg_f64"]},
        "mixed": {"ms": avg("cg_mixed_ms"), **per[-1]["cg_mixed"]},
        "mixed_over_f64_time": avg("cg_mixed_ms") / avg("cg_f64_ms"),
        "mixed_vs_f64_solution_rel_diff": per[-1]["mixed_vs_f64_rel"],
    }
    out = {
        "metric": METRIC,
        "value": round(hop_gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "48^4 SU(2) fundamental Wilson-Dirac, heat-bath-like links (plaquette 0.6), "
                               "m0=-0.3; Dslash = FP64 hopping block D_eo; CG on D^+D^ to 1e-10",
                   "dims": list(dims), "m0": m0, "tol": tol},
        "roofline": {"bound": "hbm", "achieved": round(hop_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(hop_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "hop_kernel<FUND, double> (no epilogue)",
                     "alg_bytes_per_launch": hop_alg_bytes(V, "fund", "f64")},
        "dslash": dslash,
        "cg": cg,
        "action_force_ms": avg("action_force_ms"),
    }
    if batched_ok:
        bms = avg("batched_dhat_ms")
        L, S = LINK_BYTES[("fund", "f32")], SPINOR_BYTES[("fund", "f32")]
        bbytes = V * 8 * L + (V // 2) * 5 * S * nrhs_batched
        out["batched"] = {"nrhs": nrhs_batched, "dhat_f32_ms": bms, "alg_GBs": bbytes / (bms * 1e-3) / 1e9,
                          "ms_per_rhs": bms / nrhs_batched}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_oracle_sample(U_np, psi_np, V)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
