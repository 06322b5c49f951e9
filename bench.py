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
  3. CG on D^+D^ to true residual 1e-10 in FP64 and in mixed precision
     (FP32 operator, and 16-bit operator storage: binary16 spinors with a
     per-site scale and binary16 links);
  4. the fermion-action force from the mixed solution;
  5. a batched 12-right-hand-side FP32 D^ in persistent launches (when the
     library provides it);
  6. the clover-improved operator (Sec. 2.2), Sheikholeslami-Wohlert and
     exponentiated, c_sw = 1: site-matrix build, even/odd D^_sw in FP64 and
     FP32, and CG on D^_sw^+ D^_sw in FP64 and mixed precision (FP32 and F16).

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

LINK_BYTES = {("fund", "f64"): 64, ("fund", "f32"): 32, ("fund", "f16"): 16,
              ("adj", "f64"): 72, ("adj", "f32"): 36, ("adj", "f16"): 18,
              ("fund_su2", "f64"): 32, ("fund_su2", "f32"): 16, ("fund_su2", "f16"): 8,
              ("adj_su2", "f64"): 32, ("adj_su2", "f32"): 16, ("adj_su2", "f16"): 8}
# F16 spinors: 4N binary16 complex components plus the FP32 site scale
SPINOR_BYTES = {("fund", "f64"): 128, ("fund", "f32"): 64, ("fund", "f16"): 36,
                ("adj", "f64"): 192, ("adj", "f32"): 96, ("adj", "f16"): 52,
                ("fund_su2", "f64"): 128, ("fund_su2", "f32"): 64, ("fund_su2", "f16"): 36,
                ("adj_su2", "f64"): 192, ("adj_su2", "f32"): 96, ("adj_su2", "f16"): 52}


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


def clover_site_bytes(rep, prec):
    """Packed clover field: 8 N^2 reals per site."""
    n = 2 if rep in ("fund", "fund_su2") else 3
    return 8 * n * n * (8 if prec == "f64" else 4)


def dhat_clover_alg_bytes(V, rep, prec):
    """D^_sw: the D^ bytes plus M^{-1} on odd and M on even sites, each read once."""
    return dhat_alg_bytes(V, rep, prec) + V * clover_site_bytes(rep, prec)


KERNEL_SOURCES = ["paper_2411_18511_amd/csrc/hop.h", "paper_2411_18511_amd/csrc/dslash.hip",
                  "paper_2411_18511_amd/csrc/common.h", "paper_2411_18511_amd/csrc/spin.h",
                  "paper_2411_18511_amd/csrc/clover.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hop_f64_fund_48x48x48x48.traffic.json")


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the hop kernel from the committed counter summary,
    or None when the kernel sources have changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t


def copy_ceiling(torch, dev, nbytes=1 << 30, reps=10):
    """Device-to-device copy of nbytes: the achievable read+write bandwidth on this machine."""
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"bytes_read_plus_written": 2 * nbytes, "ms": ms, "GBs": 2 * nbytes / (ms * 1e-3) / 1e9}


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


def mixed_volume_cg(torch, hrd, inputs, dev, nrhs=12, tol=1e-10):
    """12 right-hand sides on each of 16^4, 24^3x48 and 32^4, fundamental and
    adjoint (Haar links): one batched mixed-precision CG against the same 72
    systems solved one after another with the single-system mixed CG.  Timed
    once, outside the per-step figures."""
    specs = [((16, 16, 16, 16), "fund", -0.3), ((48, 24, 24, 24), "fund", -0.3), ((32, 32, 32, 32), "fund", -0.3),
             ((16, 16, 16, 16), "adj", -0.5), ((48, 24, 24, 24), "adj", -0.5), ((32, 32, 32, 32), "adj", -0.5)]
    gen = torch.Generator(device=dev)
    gen.manual_seed(4)
    probs_spec, keep = [], []
    for i, (dims, rep, m0) in enumerate(specs):
        V = int(np.prod(dims))
        n = 2 if rep == "fund" else 3
        Uf = torch.from_numpy(inputs.gauge_field(dims, 40 + i).reshape(4, V, 2, 2)).to(dev)
        Uf64 = hrd.pack_gauge(Uf, dims, "fund", "f64")
        U64 = Uf64 if rep == "fund" else hrd.represent(Uf64, dims, "f64")
        U32 = hrd.convert_gauge(U64, dims, rep)
        srcs = []
        for k in range(nrhs):
            z = torch.complex(torch.randn((V, 4, n), dtype=torch.float64, device=dev, generator=gen),
                              torch.randn((V, 4, n), dtype=torch.float64, device=dev, generator=gen)) * (0.5 ** 0.5)
            srcs.append(hrd.pack_spinor(z, dims, rep, "f64", "even"))
        src = torch.stack(srcs)
        dst = torch.zeros_like(src)
        keep.append((dims, rep, m0, U64, U32, src, dst))
        probs_spec.append({"dims": dims, "rep": rep, "nrhs": nrhs, "m0": m0, "U32": U32, "U64": U64, "src": src,
                           "dst": dst})
    probs = hrd.make_problems(probs_spec)
    work = torch.empty(hrd._lib.hrd_cg_batched_workspace_bytes(probs, len(probs)), dtype=torch.uint8, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    infos, status = hrd.cg_solve_batched(probs, tol, work=work)
    e1.record()
    e1.synchronize()
    batched_ms = e0.elapsed_time(e1)
    e0.record()
    seq_iters = []
    for dims, rep, m0, U64, U32, src, dst in keep:
        for k in range(nrhs):
            x, inf = hrd.cg_solve(U64, src[k], m0, tol, dims, rep, mode="mixed", U32=U32)
            seq_iters.append(inf["iters"])
    e1.record()
    e1.synchronize()
    seq_ms = e0.elapsed_time(e1)
    return {"problems": [f"{'x'.join(map(str, d))}/{r}" for d, r, _ in specs], "nrhs_each": nrhs,
            "status": status, "batched_ms": batched_ms, "sequential_single_ms": seq_ms,
            "speedup": seq_ms / batched_ms, "max_true_rel_residual": max(i["true_rel_residual"] for i in infos),
            "iters_batched_max": max(i["iters"] for i in infos), "iters_single_max": max(seq_iters)}


def adjoint_stage(torch, hrd, inputs, dev, dims=(32, 32, 32, 32), reps=20, tol=1e-10, m0=-0.5):
    """SU(2) with adjoint fermions on 32^4 (Haar links, m0 = -0.5): hopping block
    and even/odd D^ in FP64 / FP32 / F16 for full (ADJ) and first-row (ADJ_SU2)
    link storage, and CG to 1e-10 in every mode.  Timed once, outside the
    per-step figures."""
    V = int(np.prod(dims))
    Uf = torch.from_numpy(inputs.gauge_field(dims, 11, kind="haar").reshape(4, V, 2, 2)).to(dev)
    psi = torch.from_numpy(inputs.gaussian_spinor(dims, 3, 12).reshape(V, 4, 3)).to(dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    a, b = ev(), ev()
    out = {"dims": list(dims), "m0": m0, "links": "Haar-random SU(2)"}
    for fmt in ("adj", "adj_su2"):
        U64 = hrd.represent(hrd.pack_gauge(Uf, dims, "fund", "f64"), dims, "f64") if fmt == "adj" else \
            hrd.pack_gauge(Uf, dims, fmt, "f64")
        src_o = hrd.pack_spinor(psi, dims, fmt, "f64", "odd")
        src_e = hrd.pack_spinor(psi, dims, fmt, "f64", "even")
        r = {}
        lows = {}
        for prec in ("f64", "f32", "f16"):
            Ug = U64 if prec == "f64" else hrd.convert_gauge_prec(U64, dims, fmt, prec)
            lows[prec] = Ug
            so = hrd.convert_spinor_prec(src_o, dims, fmt, 1, "f64", prec)
            se = hrd.convert_spinor_prec(src_e, dims, fmt, 1, "f64", prec)
            dst = torch.empty_like(se)
            L, S = LINK_BYTES[(fmt, prec)], SPINOR_BYTES[(fmt, prec)]
            for kind, par, src, nrep, alg in (("hop", "hop_eo", so, reps, (V // 2) * (8 * L + 2 * S)),
                                              ("dhat", "eo", se, reps // 2, V * 8 * L + (V // 2) * 5 * S)):
                op = hrd.DiracOp(Ug, dims, fmt, prec, m0, par)
                op(src, dst)
                a.record()
                for _ in range(nrep):
                    op(src, dst)
                b.record()
                b.synchronize()
                ms = a.elapsed_time(b) / nrep
                r[f"{kind}_{prec}"] = {"ms": ms, "alg_GBs": alg / (ms * 1e-3) / 1e9,
                                       "pct_hbm_peak": 100.0 * alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            del so, se, dst
        for mode, Ulo in (("f64", None), ("mixed", lows["f32"]), ("mixed16", lows["f16"])):
            a.record()
            _, info = hrd.cg_solve(U64, src_e, m0, tol, dims, fmt, mode=mode, U32=Ulo)
            b.record()
            b.synchronize()
            r[f"cg_{mode}"] = {"ms": a.elapsed_time(b), **info}
        out[fmt] = r
        del U64, src_o, src_e, lows
    return out


SUN_LINK_BYTES = {"cplx3": 9 * 16, "cplx6": 36 * 16, "real8": 64 * 8, "su3_row2": 6 * 16}  # FP64, unpadded


def sun_stage(torch, hrd, inputs, dev, dims=(32, 32, 32, 32), reps=20, tol=1e-10, m0=-0.3):
    """SU(3) with fermions in the fundamental (CPLX3), 2-index symmetric (CPLX6)
    and adjoint (REAL8) representations: representation build, hopping block
    in FP64 / FP32 / F16 and even/odd D^ in FP32 (algorithmic bytes on
    unpadded links), and mixed / MIXED16 CG to 1e-10 for the fundamental; the
    fundamental also in the two-row format, with the clover-improved D^ (FP32)
    and MIXED16 clover CG."""
    V = int(np.prod(dims))
    Uf = inputs.gauge_field_sun(dims, 7, 3, kind="product")
    Uf_dev = torch.from_numpy(Uf.reshape(4, V, 3, 3)).to(dev)
    del Uf
    Uf64 = hrd.pack_gauge(Uf_dev, dims, "cplx3", "f64")
    del Uf_dev
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    out = {"dims": list(dims), "group": "SU(3)", "links": "products of embedded Haar SU(2) elements"}
    for rep in ("fund", "sym", "adj", "fund_row2"):
        a, b = ev(), ev()
        if rep == "fund_row2":
            # the same SU(3) links stored as two rows (third row rebuilt in the kernel)
            fmt, name = hrd.SU3_ROW2, "su3_row2"
            a.record()
            U64 = hrd.pack_gauge(hrd.unpack_gauge(Uf64, dims, "cplx3", "f64"), dims, fmt, "f64")
            b.record()
        else:
            fmt = hrd.sun_rep_format(3, rep)
            name = {hrd.CPLX3: "cplx3", hrd.CPLX6: "cplx6", hrd.REAL8: "real8"}[fmt]
            a.record()
            U64 = hrd.represent_sun(Uf64, dims, 3, rep)
            b.record()
        n = hrd.ncolour(fmt)
        b.synchronize()
        r = {"format": name, "N_R": n, "represent_ms": a.elapsed_time(b)}
        psi = torch.from_numpy(inputs.gaussian_spinor(dims, n, 8).reshape(V, 4, n)).to(dev)
        src_o = hrd.pack_spinor(psi, dims, fmt, "f64", "odd")
        src_e = hrd.pack_spinor(psi, dims, fmt, "f64", "even")
        del psi
        for prec in ("f64", "f32", "f16"):
            Ug = U64 if prec == "f64" else hrd.convert_gauge_prec(U64, dims, fmt, prec)
            so = hrd.convert_spinor_prec(src_o, dims, fmt, 1, "f64", prec)
            se = hrd.convert_spinor_prec(src_e, dims, fmt, 1, "f64", prec)
            dst = torch.empty_like(se)
            hop = hrd.DiracOp(Ug, dims, fmt, prec, m0, "hop_eo")
            hop(so, dst)
            a.record()
            for _ in range(reps):
                hop(so, dst)
            b.record()
            b.synchronize()
            ms = a.elapsed_time(b) / reps
            L = SUN_LINK_BYTES[name] // {"f64": 1, "f32": 2, "f16": 4}[prec]
            S = {"f64": 64 * n, "f32": 32 * n, "f16": 16 * n + 4}[prec]
            alg = (V // 2) * (8 * L + 2 * S)
            r[f"hop_{prec}"] = {"ms": ms, "alg_GBs": alg / (ms * 1e-3) / 1e9,
                                "pct_hbm_peak": 100.0 * alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            if prec == "f32":
                dh = hrd.DiracOp(Ug, dims, fmt, prec, m0, "eo")
                dh(se, dst)
                a.record()
                for _ in range(reps // 2):
                    dh(se, dst)
                b.record()
                b.synchronize()
                ms = a.elapsed_time(b) / (reps // 2)
                alg = V * 8 * L + (V // 2) * 5 * S
                r["dhat_f32"] = {"ms": ms, "alg_GBs": alg / (ms * 1e-3) / 1e9,
                                 "pct_hbm_peak": 100.0 * alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            if rep in ("fund", "fund_row2") and prec != "f64":
                mode = "mixed" if prec == "f32" else "mixed16"
                a.record()
                _, info = hrd.cg_solve(U64, src_e, m0, tol, dims, fmt, mode=mode, U32=Ug)
                b.record()
                b.synchronize()
                r[f"cg_{mode}"] = {"ms": a.elapsed_time(b), **info}
            del Ug, so, se, dst
        if rep in ("fund", "fund_row2"):
            a.record()
            _, info = hrd.cg_solve(U64, src_e, m0, tol, dims, fmt, mode="f64")
            b.record()
            b.synchronize()
            r["cg_f64"] = {"ms": a.elapsed_time(b), **info}
        if rep == "fund_row2":
            # clover-improved SU(3) operator (c_sw = 1): D^_sw in FP32, MIXED16 CG
            c64 = hrd.clover_build(U64, 1.0, m0, dims, fmt)
            c32 = hrd.convert_clover(c64, dims, fmt)
            U32 = hrd.convert_gauge_prec(U64, dims, fmt, "f32")
            U16 = hrd.convert_gauge_prec(U64, dims, fmt, "f16")
            se = hrd.convert_spinor_prec(src_e, dims, fmt, 1, "f64", "f32")
            dst = torch.empty_like(se)
            op = hrd.CloverOp(U32, c32, dims, fmt, "eo")
            op(se, dst)
            a.record()
            for _ in range(reps // 2):
                op(se, dst)
            b.record()
            b.synchronize()
            ms = a.elapsed_time(b) / (reps // 2)
            L, S, C = SUN_LINK_BYTES[name] // 2, 32 * n, 8 * n * n * 4
            alg = V * 8 * L + (V // 2) * 5 * S + V * C
            r["clover_dhat_f32"] = {"ms": ms, "alg_GBs": alg / (ms * 1e-3) / 1e9,
                                    "pct_hbm_peak": 100.0 * alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            a.record()
            _, info = hrd.cg_solve_clover(U64, c64, src_e, tol, dims, fmt, mode="mixed16", U32=U16, clov32=c32)
            b.record()
            b.synchronize()
            r["clover_cg_mixed16"] = {"ms": a.elapsed_time(b), **info}
            del c64, c32, U32, U16, se, dst, op
        out[rep] = r
        del U64, src_o, src_e
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--reps", type=int, default=50, help="Dslash applications timed per step")
    ap.add_argument("--dims", type=str, default="48,48,48,48")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-config4", action="store_true", help="skip the mixed-volume batched CG comparison")
    ap.add_argument("--no-sun", action="store_true", help="skip the SU(3) representations stage")
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
    LINK_FORMATS = ("fund", "fund_su2")
    CLOVER_KINDS = ("sw", "exp")
    CSW = 1.0

    def timed(fn, reps):
        a, b = ev(), ev()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps  # ms per application

    def timed_once(fn):
        a, b = ev(), ev()
        a.record()
        out = fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b), out

    def step():
        r = {}
        R = args.reps
        src_all = hrd.pack_spinor(psi_nat, dims, "fund", "f64", "all")
        src_e = hrd.pack_spinor(psi_nat, dims, "fund", "f64", "even")
        src_o = hrd.pack_spinor(psi_nat, dims, "fund", "f64", "odd")
        src_o32 = hrd.convert_spinor(src_o, dims, "fund", 1, True)
        src_e32 = hrd.convert_spinor(src_e, dims, "fund", 1, True)
        src_o16 = hrd.convert_spinor_prec(src_o, dims, "fund", 1, "f64", "f16")
        src_e16 = hrd.convert_spinor_prec(src_e, dims, "fund", 1, "f64", "f16")
        out_e16 = torch.empty_like(src_e16)
        out_e = torch.empty_like(src_e)
        out_e32 = torch.empty_like(src_e32)
        out_all = torch.empty_like(src_all)
        for fmt in LINK_FORMATS:
            # 1. gauge preparation: pack the natural links, FP32 copy
            U64 = hrd.pack_gauge(U_nat, dims, fmt, "f64")
            U32 = hrd.convert_gauge(U64, dims, fmt)
            # 2. Dslash phases, HIP events on the library's stream
            hop64 = hrd.DiracOp(U64, dims, fmt, "f64", m0, "hop_eo")
            hop32 = hrd.DiracOp(U32, dims, fmt, "f32", m0, "hop_eo")
            full64 = hrd.DiracOp(U64, dims, fmt, "f64", m0, "full")
            dhat64 = hrd.DiracOp(U64, dims, fmt, "f64", m0, "eo")
            dhatd64 = hrd.DiracOp(U64, dims, fmt, "f64", m0, "eo", dagger=True)
            dhat32 = hrd.DiracOp(U32, dims, fmt, "f32", m0, "eo")
            U16 = hrd.convert_gauge_prec(U64, dims, fmt, "f16")
            hop16 = hrd.DiracOp(U16, dims, fmt, "f16", m0, "hop_eo")
            dhat16 = hrd.DiracOp(U16, dims, fmt, "f16", m0, "eo")
            r[f"hop_f64_{fmt}"] = timed(lambda: hop64(src_o, out_e), R)
            r[f"hop_f32_{fmt}"] = timed(lambda: hop32(src_o32, out_e32), R)
            r[f"full_f64_{fmt}"] = timed(lambda: full64(src_all, out_all), R // 2)
            r[f"dhat_f64_{fmt}"] = timed(lambda: dhat64(src_e, out_e), R // 2)
            r[f"dhat_dag_f64_{fmt}"] = timed(lambda: dhatd64(src_e, out_e), R // 2)
            r[f"dhat_f32_{fmt}"] = timed(lambda: dhat32(src_e32, out_e32), R // 2)
            r[f"hop_f16_{fmt}"] = timed(lambda: hop16(src_o16, out_e16), R)
            r[f"dhat_f16_{fmt}"] = timed(lambda: dhat16(src_e16, out_e16), R // 2)
            # 3. CG solves to 1e-10 (each synchronises internally)
            r[f"cg_f64_{fmt}_ms"], (x64, i64) = timed_once(
                lambda: hrd.cg_solve(U64, src_e, m0, tol, dims, fmt, mode="f64"))
            r[f"cg_mixed_{fmt}_ms"], (xm, im) = timed_once(
                lambda: hrd.cg_solve(U64, src_e, m0, tol, dims, fmt, mode="mixed", U32=U32))
            r[f"cg_mixed16_{fmt}_ms"], (xh, ih) = timed_once(
                lambda: hrd.cg_solve(U64, src_e, m0, tol, dims, fmt, mode="mixed16", U32=U16))
            r[f"cg_f64_{fmt}"], r[f"cg_mixed_{fmt}"], r[f"cg_mixed16_{fmt}"] = i64, im, ih
            n64 = hrd.blas_norm2(x64, dims, fmt, "f64", 1)
            d = xm.clone()
            hrd.blas_axpy(-1.0, x64, d, dims, fmt, "f64", 1)
            r[f"mixed_vs_f64_rel_{fmt}"] = float(np.sqrt(hrd.blas_norm2(d, dims, fmt, "f64", 1) / n64))
            d = xh.clone()
            hrd.blas_axpy(-1.0, x64, d, dims, fmt, "f64", 1)
            r[f"mixed16_vs_f64_rel_{fmt}"] = float(np.sqrt(hrd.blas_norm2(d, dims, fmt, "f64", 1) / n64))
            # 4. fermion force from the mixed solution
            r[f"action_force_{fmt}_ms"], _ = timed_once(lambda: hrd.action_force(U64, xm, m0, dims, fmt))
            # 5. batched multi-RHS D^ (FP32)
            if batched_ok:
                srcs = torch.stack([hrd.convert_spinor(hrd.pack_spinor(t, dims, fmt, "f64", "even"), dims, fmt,
                                                       1, True) for t in rhs_nat])
                dsts = torch.empty_like(srcs)
                probs = hrd.make_problems([{"dims": dims, "rep": fmt, "nrhs": nrhs_batched, "m0": m0, "U32": U32,
                                            "src": srcs, "dst": dsts}])
                wb = torch.empty(max(hrd.batched_workspace_bytes(probs, "eo"), 1), dtype=torch.uint8, device=dev)
                r[f"batched_dhat_{fmt}"] = timed(lambda: hrd.dirac_apply_batched(probs, "eo", tune=tunes[fmt],
                                                                                 work=wb), 5)
                del srcs, dsts, wb
            # 6. clover-improved operator (fundamental links only)
            if fmt == "fund":
                for kind in CLOVER_KINDS:
                    r[f"clover_build_{kind}_ms"], c64 = timed_once(
                        lambda: hrd.clover_build(U64, CSW, m0, dims, fmt, kind=kind))
                    c32 = hrd.convert_clover(c64, dims, fmt)
                    cd64 = hrd.CloverOp(U64, c64, dims, fmt, "eo")
                    cd32 = hrd.CloverOp(U32, c32, dims, fmt, "eo")
                    r[f"dhat_clover_{kind}_f64"] = timed(lambda: cd64(src_e, out_e), R // 2)
                    r[f"dhat_clover_{kind}_f32"] = timed(lambda: cd32(src_e32, out_e32), R // 2)
                    r[f"cg_clover_{kind}_f64_ms"], (_, ic64) = timed_once(
                        lambda: hrd.cg_solve_clover(U64, c64, src_e, tol, dims, fmt, mode="f64"))
                    r[f"cg_clover_{kind}_mixed_ms"], (_, icm) = timed_once(
                        lambda: hrd.cg_solve_clover(U64, c64, src_e, tol, dims, fmt, mode="mixed", U32=U32,
                                                    clov32=c32))
                    r[f"cg_clover_{kind}_mixed16_ms"], (_, ich) = timed_once(
                        lambda: hrd.cg_solve_clover(U64, c64, src_e, tol, dims, fmt, mode="mixed16", U32=U16,
                                                    clov32=c32))
                    r[f"cg_clover_{kind}_f64"], r[f"cg_clover_{kind}_mixed"] = ic64, icm
                    r[f"cg_clover_{kind}_mixed16"] = ich
                    del c64, c32, cd64, cd32
            del U64, U32, U16, x64, xm, xh, d
        return r

    ceiling = copy_ceiling(torch, dev)
    tunes = {}
    if batched_ok:
        # launch shape of the batched stages, chosen by the library's autotuner (untimed setup)
        for fmt in LINK_FORMATS:
            U32t = hrd.convert_gauge(hrd.pack_gauge(U_nat, dims, fmt, "f64"), dims, fmt)
            srcs = torch.zeros((nrhs_batched, hrd.spinor_bytes(dims, fmt, "f32", 1)), dtype=torch.uint8, device=dev)
            probs = hrd.make_problems([{"dims": dims, "rep": fmt, "nrhs": nrhs_batched, "m0": m0, "U32": U32t,
                                        "src": srcs, "dst": torch.zeros_like(srcs)}])
            tunes[fmt] = hrd.autotune_batched(probs)
            print(f"[bench] batched tune {fmt}: {tunes[fmt]}", file=sys.stderr, flush=True)
            del U32t, srcs, probs
    for w in range(args.warmup):
        print(f"[bench] warmup {w}", file=sys.stderr, flush=True)
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = []
    for s_ in range(args.steps):
        per.append(step())
        p = per[-1]
        print(f"[bench] step {s_} done: hop f64 {p['hop_f64_fund']:.3f} ms, cg f64 {p['cg_f64_fund_ms']:.1f} ms, "
              f"cg mixed {p['cg_mixed_fund_ms']:.1f} ms, cg mixed su2 {p['cg_mixed_fund_su2_ms']:.1f} ms, "
              f"cg mixed16 su2 {p['cg_mixed16_fund_su2_ms']:.1f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    def avg(k):
        return float(np.mean([p[k] for p in per]))

    dslash = {}
    for fmt in LINK_FORMATS:
        for key, fn, prec in [("hop_f64", hop_alg_bytes, "f64"), ("hop_f32", hop_alg_bytes, "f32"),
                              ("full_f64", full_alg_bytes, "f64"), ("dhat_f64", dhat_alg_bytes, "f64"),
                              ("dhat_dag_f64", dhat_alg_bytes, "f64"), ("dhat_f32", dhat_alg_bytes, "f32"),
                              ("hop_f16", hop_alg_bytes, "f16"), ("dhat_f16", dhat_alg_bytes, "f16")]:
            ms = avg(f"{key}_{fmt}")
            sites = V // 2 if key.startswith("hop") else V
            gbs = fn(V, fmt, prec) / (ms * 1e-3) / 1e9
            dslash[f"{key}_{fmt}"] = {"ms": ms, "alg_GBs": gbs, "pct_hbm_peak": 100.0 * gbs / HBM_PEAK_GBS,
                                      "site_updates_per_s": sites / (ms * 1e-3),
                                      "alg_bytes": fn(V, fmt, prec)}
    cg = {}
    for fmt in LINK_FORMATS:
        cg[fmt] = {
            "f64": {"ms": avg(f"cg_f64_{fmt}_ms"), **per[-1][f"cg_f64_{fmt}"]},
            "mixed": {"ms": avg(f"cg_mixed_{fmt}_ms"), **per[-1][f"cg_mixed_{fmt}"]},
            "mixed16": {"ms": avg(f"cg_mixed16_{fmt}_ms"), **per[-1][f"cg_mixed16_{fmt}"]},
            "mixed_over_f64_time": avg(f"cg_mixed_{fmt}_ms") / avg(f"cg_f64_{fmt}_ms"),
            "mixed16_over_f64_time": avg(f"cg_mixed16_{fmt}_ms") / avg(f"cg_f64_{fmt}_ms"),
            "mixed_vs_f64_solution_rel_diff": per[-1][f"mixed_vs_f64_rel_{fmt}"],
            "mixed16_vs_f64_solution_rel_diff": per[-1][f"mixed16_vs_f64_rel_{fmt}"],
            "action_force_ms": avg(f"action_force_{fmt}_ms"),
        }
    clover = {"csw": CSW, "rep": "fund"}
    for kind in CLOVER_KINDS:
        d_ = {"build_ms": avg(f"clover_build_{kind}_ms")}
        for prec in ("f64", "f32"):
            ms = avg(f"dhat_clover_{kind}_{prec}")
            gbs = dhat_clover_alg_bytes(V, "fund", prec) / (ms * 1e-3) / 1e9
            d_[f"dhat_{prec}"] = {"ms": ms, "alg_GBs": gbs, "pct_hbm_peak": 100.0 * gbs / HBM_PEAK_GBS,
                                  "alg_bytes": dhat_clover_alg_bytes(V, "fund", prec),
                                  "over_wilson_dhat": ms / avg(f"dhat_{prec}_fund")}
        d_["cg_f64"] = {"ms": avg(f"cg_clover_{kind}_f64_ms"), **per[-1][f"cg_clover_{kind}_f64"]}
        d_["cg_mixed"] = {"ms": avg(f"cg_clover_{kind}_mixed_ms"), **per[-1][f"cg_clover_{kind}_mixed"]}
        d_["cg_mixed16"] = {"ms": avg(f"cg_clover_{kind}_mixed16_ms"), **per[-1][f"cg_clover_{kind}_mixed16"]}
        d_["mixed_over_f64_time"] = d_["cg_mixed"]["ms"] / d_["cg_f64"]["ms"]
        d_["mixed16_over_f64_time"] = d_["cg_mixed16"]["ms"] / d_["cg_f64"]["ms"]
        clover[kind] = d_
    hop = dslash["hop_f64_fund"]
    hop_gbs = hop["alg_GBs"]
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
                               "m0=-0.3; Dslash = FP64 hopping block D_eo with full 2x2 links; CG on D^+D^ "
                               "to 1e-10 in FP64 and mixed precision, full and first-row SU(2) link storage",
                   "dims": list(dims), "m0": m0, "tol": tol},
        "roofline": {"bound": "hbm", "achieved": round(hop_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(hop_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "hop_kernel<FUND, double, dagger=false, no epilogue>",
                     "alg_bytes_per_launch": hop_alg_bytes(V, "fund", "f64"), "avg_launch_ms": hop["ms"]},
        "dslash": dslash,
        "cg": cg,
        "clover": clover,
        "copy_ceiling": ceiling,
    }
    tr = measured_traffic()
    if tr is not None:
        out["roofline"]["traffic"] = tr["bytes_per_launch"]
        out["roofline"]["traffic_source"] = tr["source"]
    if batched_ok:
        out["batched"] = {}
        for fmt in LINK_FORMATS:
            bms = avg(f"batched_dhat_{fmt}")
            L, S = LINK_BYTES[(fmt, "f32")], SPINOR_BYTES[(fmt, "f32")]
            bbytes = V * 8 * L + (V // 2) * 5 * S * nrhs_batched
            out["batched"][fmt] = {"nrhs": nrhs_batched, "dhat_f32_ms": bms, "alg_GBs": bbytes / (bms * 1e-3) / 1e9,
                                   "ms_per_rhs": bms / nrhs_batched, "tune": tunes[fmt],
                                   "single_dhat_f32_ms": avg(f"dhat_f32_{fmt}")}
    if batched_ok and not args.no_config4:
        out["batched_cg_mixed_volumes"] = mixed_volume_cg(torch, hrd, inputs, dev)
    if not args.no_sun:
        print("[bench] SU(2) adjoint stage", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_stage(torch, hrd, inputs, dev)
        print("[bench] SU(3) representations stage", file=sys.stderr, flush=True)
        out["sun"] = sun_stage(torch, hrd, inputs, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_oracle_sample(U_np, psi_np, V)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
