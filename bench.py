"""Benchmark of the single-GPU hot path on the 48^4 SU(2) workload.

Workload (the paper's per-GPU weak-scaling share, Table 1): a 48^4 lattice,
SU(2) fundamental fermions, heat-bath-like links (mean plaquette 0.6),
m0 = -0.3, Gaussian complex128 source; synthetic seeded inputs, resident in
HBM before timing starts.

One step = one pass over every stage of the hot path:
  1. gauge preparation: pack the natural links, FP32 and F16 copies;
  2. the Dslash: R applications each of the hopping block D_eo, the plain D
     and the even/odd D^ (and dagger) in FP64, FP32 and F16, timed with HIP
     events on the library's stream;
  3. CG on D^+D^ to true residual 1e-10 in FP64 and in mixed precision
     (FP32 operator, and 16-bit operator storage: binary16 spinors with a
     per-site scale and binary16 links);
  4. the fermion-action force from the mixed solution;
  5. a batched 12-right-hand-side FP32 D^ in persistent launches;
  6. the clover-improved operator (Sec. 2.2), Sheikholeslami-Wohlert and
     exponentiated, c_sw = 1: site-matrix build, even/odd D^_sw in FP64 and
     FP32, and CG on D^_sw^+ D^_sw in FP64 and mixed precision (FP32 and F16);
for full and first-row link storage.  After the steps, once each: the
bandwidth ceiling (stream probes), the adjoint representation at 48^4, the
mixed-volume batched CG, the adjoint and SU(3) stages at 32^4, the SU(4)
stage at 24^4, and the CPU
oracle (timings and the error of each GPU solution against the oracle's
FP64 solution).

Every timed section is bracketed by two one-block marker launches outside
its HIP-event window, and `--manifest` writes the list of sections, so that a
rocprofv3 kernel trace or counter run of the same command splits into the
same sections (`--summarize` turns those runs into the summaries under
profiles/, which later runs read back when the library sources match).

Prints one JSON line.  `value` is the FP64 Dslash (hopping block) bandwidth
on algorithmic bytes: each link, each source spinor and each output spinor
counted once per application.
"""
import argparse
import csv
import glob
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "Dslash GB/s & %HBM peak at 48^4 SU(2); mixed vs FP64 CG time to 1e-10"
SECTIONS_FILE = os.path.join(ROOT, "profiles", "bench_48x48x48x48_sections.json")

LINK_BYTES = {("fund", "f64"): 64, ("fund", "f32"): 32, ("fund", "f16"): 16,
              ("adj", "f64"): 72, ("adj", "f32"): 36, ("adj", "f16"): 18,
              ("fund_su2", "f64"): 32, ("fund_su2", "f32"): 16, ("fund_su2", "f16"): 8,
              ("adj_su2", "f64"): 32, ("adj_su2", "f32"): 16, ("adj_su2", "f16"): 8}
# F16 spinors: 4N binary16 complex components plus the FP32 site scale
SPINOR_BYTES = {("fund", "f64"): 128, ("fund", "f32"): 64, ("fund", "f16"): 36,
                ("adj", "f64"): 192, ("adj", "f32"): 96, ("adj", "f16"): 52,
                ("fund_su2", "f64"): 128, ("fund_su2", "f32"): 64, ("fund_su2", "f16"): 36,
                ("adj_su2", "f64"): 192, ("adj_su2", "f32"): 96, ("adj_su2", "f16"): 52}


# ---------------------------------------------------------------------------
# byte counts (L = link bytes, S = spinor bytes per site)
#   algorithmic ("alg"): each link, source and output spinor once per application
#   conventional ("conv", the paper's per-access count): every link and every
#   neighbour spinor read at every target site, plus the centre and the output
# ---------------------------------------------------------------------------

def _ls(rep, prec):
    return LINK_BYTES[(rep, prec)], SPINOR_BYTES[(rep, prec)]


def hop_alg_bytes(V, rep, prec):
    """One hopping-block application (V/2 target sites): 8 links, the source
    spinor and the output spinor per target site."""
    L, S = _ls(rep, prec)
    return (V // 2) * (8 * L + 2 * S)


def hop_conv_bytes(V, rep, prec):
    L, S = _ls(rep, prec)
    return (V // 2) * (8 * L + 9 * S)


def full_alg_bytes(V, rep, prec):
    """Plain D on all V sites: each link once, psi and out once."""
    L, S = _ls(rep, prec)
    return V * (4 * L + 2 * S)


def full_conv_bytes(V, rep, prec):
    L, S = _ls(rep, prec)
    return V * (8 * L + 10 * S)


def dhat_alg_bytes(V, rep, prec):
    """D^ = two hops plus the m*psi read of the second: V (8L + 2.5 S)."""
    L, S = _ls(rep, prec)
    return V * (8 * L) + (V // 2) * 5 * S


def dhat_conv_bytes(V, rep, prec):
    L, S = _ls(rep, prec)
    return (V // 2) * (8 * L + 9 * S) + (V // 2) * (8 * L + 10 * S)


def clover_site_bytes(rep, prec):
    """Packed clover field: 8 N^2 reals per site."""
    n = 2 if rep in ("fund", "fund_su2") else 3
    return 8 * n * n * (8 if prec == "f64" else 4)


def dhat_clover_alg_bytes(V, rep, prec):
    """D^_sw: the D^ bytes plus M^{-1} on odd and M on even sites, each read once."""
    return dhat_alg_bytes(V, rep, prec) + V * clover_site_bytes(rep, prec)


OPS = {"hop": (hop_alg_bytes, hop_conv_bytes, 1, 0.5), "full": (full_alg_bytes, full_conv_bytes, 1, 1.0),
       "dhat": (dhat_alg_bytes, dhat_conv_bytes, 2, 1.0)}


# ---------------------------------------------------------------------------
# timed sections and their markers
# ---------------------------------------------------------------------------

class Sections:
    """Ordered record of the timed sections of a run.  Each section is
    bracketed by a one-block stream-probe launch before and after its event
    window; `--summarize` splits a kernel trace of the same command at those
    marker dispatches and assigns the pieces to the sections in order."""

    def __init__(self, torch, hrd, dev):
        self.torch, self.hrd = torch, hrd
        self.entries = []
        self._msrc = torch.zeros(32, dtype=torch.uint8, device=dev)
        self._mdst = torch.zeros(16, dtype=torch.uint8, device=dev)

    def mark(self):
        self.hrd.stream_probe(self._msrc, self._mdst, 16, 16, tiled=False)

    def _events(self):
        return self.torch.cuda.Event(enable_timing=True), self.torch.cuda.Event(enable_timing=True)

    def timed(self, name, fn, reps, launches=None, alg=None, conv=None, sites=None):
        """ms per application of fn over reps back-to-back applications."""
        a, b = self._events()
        self.mark()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        self.mark()
        b.synchronize()
        ms = a.elapsed_time(b) / reps
        self.entries.append({"name": name, "reps": reps, "launches": launches, "alg_bytes": alg,
                             "conv_bytes": conv, "sites": sites, "ms": ms})
        return ms

    def timed_once(self, name, fn):
        a, b = self._events()
        self.mark()
        a.record()
        out = fn()
        b.record()
        self.mark()
        b.synchronize()
        ms = a.elapsed_time(b)
        self.entries.append({"name": name, "reps": 1, "launches": None, "alg_bytes": None, "conv_bytes": None,
                             "sites": None, "ms": ms})
        return ms, out

    def op(self, name, fn, reps, V, rep, prec, kind):
        alg_f, conv_f, launches, site_frac = OPS[kind]
        return self.timed(name, fn, reps, launches, alg_f(V, rep, prec), conv_f(V, rep, prec), int(V * site_frac))


def dslash_entry(ms, alg, conv, sites):
    gbs = alg / (ms * 1e-3) / 1e9
    return {"ms": ms, "alg_GBs": gbs, "pct_hbm_peak": 100.0 * gbs / HBM_PEAK_GBS,
            "conv_GBs": conv / (ms * 1e-3) / 1e9, "site_updates_per_s": sites / (ms * 1e-3), "alg_bytes": alg,
            "conv_bytes": conv}


# ---------------------------------------------------------------------------
# committed counter summaries (read back only while the library sources match)
# ---------------------------------------------------------------------------

def load_sections_summary(build_hash):
    if not os.path.exists(SECTIONS_FILE):
        return None
    with open(SECTIONS_FILE) as f:
        s = json.load(f)
    if s.get("source_hash") != build_hash:
        return None
    return s


def attach_measured(entry, name, summ):
    """Add the profiled duration and the calibrated HBM bytes of section `name`."""
    if summ is None or name not in summ["sections"]:
        return
    m = summ["sections"][name]
    if m.get("rocprof_ms") is not None:
        entry["rocprof_ms"] = m["rocprof_ms"]
        if entry.get("alg_bytes"):
            entry["alg_GBs_at_rocprof_ms"] = entry["alg_bytes"] / (m["rocprof_ms"] * 1e-3) / 1e9
    if m.get("traffic_bytes") is not None:
        entry["traffic_bytes"] = m["traffic_bytes"]
        entry["traffic_over_alg"] = m.get("traffic_over_alg")
        entry["dram_GBs"] = m["traffic_bytes"] / (entry["ms"] * 1e-3) / 1e9
        entry["dram_pct_hbm_peak"] = 100.0 * entry["dram_GBs"] / HBM_PEAK_GBS


# ---------------------------------------------------------------------------
# bandwidth ceiling: stream probes with the kernels' access instructions
# ---------------------------------------------------------------------------

PROBES = [("probe_copy", 1, False), ("probe_r5w1_tiled", 5, True), ("probe_r5w1_planes", 5, False),
          ("probe_r16w1_tiled", 16, True)]


def stream_ceiling(torch, hrd, rec, dev, write_bytes=512 << 20, reps=10):
    """Read/write mixes streamed by hrd_stream_probe: a copy (1:1), the hop's
    mix (5 reads per write: 8L + S read, S written per target site for FP64
    and FP32 fundamental links) in the tiled and the plane layout, and a
    read-mostly 16:1 mix."""
    kmax = max(k for _, k, _ in PROBES)
    src = torch.empty(kmax * write_bytes, dtype=torch.uint8, device=dev)
    src.fill_(1)
    dst = torch.empty(write_bytes, dtype=torch.uint8, device=dev)
    out = {}
    for name, k, tiled in PROBES:
        rb = k * write_bytes
        hrd.stream_probe(src, dst, rb, write_bytes, tiled)
        ms = rec.timed(name, lambda: hrd.stream_probe(src, dst, rb, write_bytes, tiled), reps, 1, rb + write_bytes,
                       rb + write_bytes)
        gbs = (rb + write_bytes) / (ms * 1e-3) / 1e9
        out[name] = {"read_bytes": rb, "write_bytes": write_bytes, "read_fraction": k / (k + 1.0),
                     "layout": "64-element tiles" if tiled else "one array per plane", "ms": ms, "GBs": gbs,
                     "pct_hbm_peak": 100.0 * gbs / HBM_PEAK_GBS}
    del src, dst
    return out


# ---------------------------------------------------------------------------
# CPU oracle: timings on the host cores, and the error of the GPU solutions
# ---------------------------------------------------------------------------

def cpu_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    threads = int(os.environ.get("OMP_NUM_THREADS", nproc))
    return model, nproc, threads


def _median_time(fn, n=3):
    ts = []
    for _ in range(n):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def cpu_oracle_baseline(U_np, psi_np, V, budget_s=10.0):
    """The oracle's hopping term (target parity even) on the full 48^4 lattice,
    repeated for budget_s: the reported `value` of the CPU baseline."""
    import oracle as O

    O._load()
    _, _, threads = cpu_info()
    n = 0
    t0 = time.perf_counter()
    while True:
        O.hopping(U_np, psi_np, 1)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            break
    gbs = n * hop_alg_bytes(V, "fund", "f64") / dt / 1e9
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} FP64 hopping-block applications (even targets) of the oracle on the full "
                      f"{'x'.join(map(str, U_np.shape[1:5]))} fundamental lattice in {dt:.1f} s, "
                      f"same algorithmic byte count per application as the GPU figure"}


def cpu_oracle_configs(inputs, U48, psi48, m0_48, with_cg=True):
    """Oracle timings per parity configuration: D and D^ (median of 3) on 8^4
    fund, 32^4 adjoint and 48^4 fund; the oracle CG to 1e-10 on 8^4 fund
    (numpy iteration) and 32^4 adjoint (the same iteration in C); the force on
    24^3x48 adjoint links."""
    import oracle as O

    out = {}
    cfgs = [("c1_8^4_fund", (8, 8, 8, 8), "fund", -0.2, 1), ("c2_32^4_adj", (32, 32, 32, 32), "adj", -0.5, 2),
            ("c3_48^4_fund", None, "fund", m0_48, 3)]
    for name, dims, rep, m0, seed in cfgs:
        if dims is None:
            U, psi, dims = U48, psi48, tuple(psi48.shape[:4])
        else:
            U = inputs.gauge_field(dims, seed, kind="haar")
            if rep == "adj":
                U = O.represent_adjoint(U)
            psi = inputs.gaussian_spinor(dims, U.shape[-1], 10 + seed)
        V = int(np.prod(dims))
        lrep = "fund" if rep == "fund" else "adj"
        psi_e = O.restrict(psi, 0)
        t_d = _median_time(lambda: O.dirac(U, psi, m0))
        t_dh = _median_time(lambda: O.dhat(U, psi_e, m0))
        r = {"dims": list(dims), "rep": rep, "m0": m0,
             "D_ms": 1e3 * t_d, "D_site_updates_per_s": V / t_d,
             "D_alg_GBs": full_alg_bytes(V, lrep, "f64") / t_d / 1e9,
             "Dhat_ms": 1e3 * t_dh, "Dhat_site_updates_per_s": V / t_dh,
             "Dhat_alg_GBs": dhat_alg_bytes(V, lrep, "f64") / t_dh / 1e9}
        if with_cg and name == "c1_8^4_fund":
            t0 = time.perf_counter()
            _, info = O.cg(U, psi_e, m0, 1e-10)
            r["cg"] = {"impl": "oracle.cg (numpy)", "seconds": time.perf_counter() - t0, **info}
        if with_cg and name == "c2_32^4_adj":
            t0 = time.perf_counter()
            _, info = O.cg_native(U, psi_e, m0, 1e-10, progress=20)
            r["cg"] = {"impl": "oracle.cg_native (C)", "seconds": time.perf_counter() - t0, **info}
        out[name] = r
        del U, psi, psi_e
    dims5 = (48, 24, 24, 24)
    U5 = O.represent_adjoint(inputs.gauge_field(dims5, 5, kind="haar"))
    X = inputs.gaussian_spinor(dims5, 3, 51)
    Y = inputs.gaussian_spinor(dims5, 3, 52)
    t_f = _median_time(lambda: O.force(X, Y, real_links=True))
    out["c5_24^3x48_adj_force"] = {"dims": list(dims5), "seconds": t_f,
                                   "site_updates_per_s": int(np.prod(dims5)) / t_f}
    del U5, X, Y
    return out


def oracle_solution_errors(U48, b48, m0, sols, tol=1e-12):
    """Solve A x = b with the oracle's CG (C iteration, FP64, from x = 0) to
    tol, then state for every GPU solution ||x - x_oracle|| / ||x_oracle|| and
    its true residual recomputed by the oracle."""
    import oracle as O

    t0 = time.perf_counter()
    x_orc, info = O.cg_native(U48, b48, m0, tol, progress=20)
    out = {"oracle_cg": {"tol": tol, "seconds": time.perf_counter() - t0, **info}, "solutions": {}}
    nx = np.linalg.norm(x_orc)
    for key, x in sols.items():
        out["solutions"][key] = {"rel_error_vs_oracle": float(np.linalg.norm(x - x_orc) / nx),
                                 "oracle_true_rel_residual": float(O.true_residual_native(U48, b48, x, m0))}
    return out


# ---------------------------------------------------------------------------
# once-after stages
# ---------------------------------------------------------------------------

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


def adjoint48_stage(torch, hrd, inputs, rec, summ, U_nat, dims, m0=-0.3, reps=20):
    """SU(2) adjoint fermions on the 48^4 links of the workload: hopping block,
    plain D and D^ in FP64 / FP32 / F16 for full (ADJ) and first-row (ADJ_SU2)
    link storage, as timed sections."""
    V = int(np.prod(dims))
    psi = torch.from_numpy(inputs.gaussian_spinor(dims, 3, 48).reshape(V, 4, 3)).to(U_nat.device)
    out = {}
    for fmt in ("adj", "adj_su2"):
        Uf64 = hrd.pack_gauge(U_nat, dims, "fund", "f64") if fmt == "adj" else None
        U64 = hrd.represent(Uf64, dims, "f64") if fmt == "adj" else hrd.pack_gauge(U_nat, dims, fmt, "f64")
        del Uf64
        src_all = hrd.pack_spinor(psi, dims, fmt, "f64", "all")
        src_o = hrd.pack_spinor(psi, dims, fmt, "f64", "odd")
        src_e = hrd.pack_spinor(psi, dims, fmt, "f64", "even")
        for prec in ("f64", "f32", "f16"):
            Ug = U64 if prec == "f64" else hrd.convert_gauge_prec(U64, dims, fmt, prec)
            sa = hrd.convert_spinor_prec(src_all, dims, fmt, 2, "f64", prec) if prec != "f64" else src_all
            so = hrd.convert_spinor_prec(src_o, dims, fmt, 1, "f64", prec) if prec != "f64" else src_o
            se = hrd.convert_spinor_prec(src_e, dims, fmt, 1, "f64", prec) if prec != "f64" else src_e
            da, dh = torch.empty_like(sa), torch.empty_like(se)
            for kind, par, src, dst, nrep in (("hop", "hop_eo", so, dh, reps), ("full", "full", sa, da, reps // 2),
                                             ("dhat", "eo", se, dh, reps // 2)):
                opx = hrd.DiracOp(Ug, dims, fmt, prec, m0, par)
                opx(src, dst)
                name = f"{kind}_{prec}_{fmt}"
                ms = rec.op(name, lambda: opx(src, dst), nrep, V, fmt, prec, kind)
                e = dslash_entry(ms, OPS[kind][0](V, fmt, prec), OPS[kind][1](V, fmt, prec), int(V * OPS[kind][3]))
                attach_measured(e, name, summ)
                out[name] = e
            del Ug, sa, so, se, da, dh
        del U64, src_all, src_o, src_e
    return out


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
            for kind, par, src, nrep in (("hop", "hop_eo", so, reps), ("dhat", "eo", se, reps // 2)):
                op = hrd.DiracOp(Ug, dims, fmt, prec, m0, par)
                op(src, dst)
                a.record()
                for _ in range(nrep):
                    op(src, dst)
                b.record()
                b.synchronize()
                ms = a.elapsed_time(b) / nrep
                alg = OPS[kind][0](V, fmt, prec)
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


SUN_LINK_BYTES = {"cplx3": 9 * 16, "cplx4": 16 * 16, "cplx6": 36 * 16, "cplx10": 100 * 16, "real8": 64 * 8,
                  "real15": 225 * 8, "su3_row2": 6 * 16}  # FP64, unpadded
SUN_FORMAT_NAMES = {"cplx3": "CPLX3", "cplx4": "CPLX4", "cplx6": "CPLX6", "cplx10": "CPLX10", "real8": "REAL8",
                    "real15": "REAL15"}


def sun_stage(torch, hrd, inputs, dev, dims=(32, 32, 32, 32), reps=20, tol=1e-10, m0=-0.3, nc=3):
    """SU(nc) fermions in the fundamental and higher representations: the
    representation build, hopping block in FP64 / FP32 / F16 and even/odd D^
    in FP32 (algorithmic bytes on unpadded links) for every representation.
    SU(3) (fundamental CPLX3, 2-index symmetric CPLX6, adjoint REAL8): mixed /
    MIXED16 / FP64 CG to 1e-10 for the fundamental, which also runs in the
    two-row format with the clover-improved D^ (FP32) and MIXED16 clover CG.
    SU(4) (fundamental CPLX4, antisymmetric CPLX6, symmetric CPLX10, adjoint
    REAL15): MIXED16 CG to 1e-10 for every representation, FP64 CG for the
    fundamental."""
    V = int(np.prod(dims))
    Uf = inputs.gauge_field_sun(dims, 7, nc, kind="product")
    Uf_dev = torch.from_numpy(Uf.reshape(4, V, nc, nc)).to(dev)
    del Uf
    ffmt = "cplx3" if nc == 3 else "cplx4"
    Uf64 = hrd.pack_gauge(Uf_dev, dims, ffmt, "f64")
    del Uf_dev
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    out = {"dims": list(dims), "group": f"SU({nc})", "links": "products of embedded Haar SU(2) elements"}
    reps_list = ("fund", "sym", "adj", "fund_row2") if nc == 3 else ("fund", "asym", "sym", "adj")
    for rep in reps_list:
        a, b = ev(), ev()
        if rep == "fund_row2":
            # the same SU(3) links stored as two rows (third row rebuilt in the kernel)
            fmt, name = hrd.SU3_ROW2, "su3_row2"
            a.record()
            U64 = hrd.pack_gauge(hrd.unpack_gauge(Uf64, dims, "cplx3", "f64"), dims, fmt, "f64")
            b.record()
        else:
            fmt = hrd.sun_rep_format(nc, rep)
            name = next(k for k, v in SUN_FORMAT_NAMES.items() if getattr(hrd, v) == fmt)
            a.record()
            U64 = hrd.represent_sun(Uf64, dims, nc, rep)
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
            if (rep in ("fund", "fund_row2") and prec != "f64") or (nc == 4 and prec == "f16"):
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


# ---------------------------------------------------------------------------
# the benchmark
# ---------------------------------------------------------------------------

def run(args):
    import torch

    import __graft_entry__  # noqa: F401  (puts the repo root on sys.path)
    from paper_2411_18511_amd import hrd, inputs

    dims = tuple(int(x) for x in args.dims.split(","))
    V = int(np.prod(dims))
    m0, tol = -0.3, 1e-10
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    summ = load_sections_summary(hrd.build_hash())
    rec = Sections(torch, hrd, dev)

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

    LINK_FORMATS = ("fund", "fund_su2")
    CLOVER_KINDS = ("sw", "exp")
    CSW = 1.0
    keep_solutions = {}

    def step(last):
        r = {}
        R = args.reps
        src_all = hrd.pack_spinor(psi_nat, dims, "fund", "f64", "all")
        src_e = hrd.pack_spinor(psi_nat, dims, "fund", "f64", "even")
        src_o = hrd.pack_spinor(psi_nat, dims, "fund", "f64", "odd")
        lo = {p: {"all": hrd.convert_spinor_prec(src_all, dims, "fund", 2, "f64", p),
                  "e": hrd.convert_spinor_prec(src_e, dims, "fund", 1, "f64", p),
                  "o": hrd.convert_spinor_prec(src_o, dims, "fund", 1, "f64", p)} for p in ("f32", "f16")}
        lo["f64"] = {"all": src_all, "e": src_e, "o": src_o}
        outs = {p: {"all": torch.empty_like(lo[p]["all"]), "e": torch.empty_like(lo[p]["e"])} for p in lo}
        for fmt in LINK_FORMATS:
            # 1. gauge preparation: pack the natural links, FP32 and F16 copies
            U64 = hrd.pack_gauge(U_nat, dims, fmt, "f64")
            U32 = hrd.convert_gauge(U64, dims, fmt)
            U16 = hrd.convert_gauge_prec(U64, dims, fmt, "f16")
            Us = {"f64": U64, "f32": U32, "f16": U16}
            # 2. Dslash phases, HIP events on the library's stream
            for prec in ("f64", "f32", "f16"):
                for kind, par, sk, ok, nrep in (("hop", "hop_eo", "o", "e", R), ("full", "full", "all", "all", R // 2),
                                                ("dhat", "eo", "e", "e", R // 2)):
                    opx = hrd.DiracOp(Us[prec], dims, fmt, prec, m0, par)
                    s_, d_ = lo[prec][sk], outs[prec][ok]
                    r[f"{kind}_{prec}_{fmt}"] = rec.op(f"{kind}_{prec}_{fmt}", lambda: opx(s_, d_), nrep, V, fmt,
                                                       prec, kind)
            dd = hrd.DiracOp(U64, dims, fmt, "f64", m0, "eo", dagger=True)
            r[f"dhat_dag_f64_{fmt}"] = rec.op(f"dhat_dag_f64_{fmt}", lambda: dd(src_e, outs["f64"]["e"]), R // 2, V,
                                              fmt, "f64", "dhat")
            # 3. CG solves to 1e-10 (each synchronises internally)
            r[f"cg_f64_{fmt}_ms"], (x64, i64) = rec.timed_once(
                f"cg_f64_{fmt}", lambda: hrd.cg_solve(U64, src_e, m0, tol, dims, fmt, mode="f64"))
            r[f"cg_mixed_{fmt}_ms"], (xm, im) = rec.timed_once(
                f"cg_mixed_{fmt}", lambda: hrd.cg_solve(U64, src_e, m0, tol, dims, fmt, mode="mixed", U32=U32))
            r[f"cg_mixed16_{fmt}_ms"], (xh, ih) = rec.timed_once(
                f"cg_mixed16_{fmt}", lambda: hrd.cg_solve(U64, src_e, m0, tol, dims, fmt, mode="mixed16", U32=U16))
            r[f"cg_f64_{fmt}"], r[f"cg_mixed_{fmt}"], r[f"cg_mixed16_{fmt}"] = i64, im, ih
            n64 = hrd.blas_norm2(x64, dims, fmt, "f64", 1)
            d = xm.clone()
            hrd.blas_axpy(-1.0, x64, d, dims, fmt, "f64", 1)
            r[f"mixed_vs_f64_rel_{fmt}"] = float(np.sqrt(hrd.blas_norm2(d, dims, fmt, "f64", 1) / n64))
            d = xh.clone()
            hrd.blas_axpy(-1.0, x64, d, dims, fmt, "f64", 1)
            r[f"mixed16_vs_f64_rel_{fmt}"] = float(np.sqrt(hrd.blas_norm2(d, dims, fmt, "f64", 1) / n64))
            if last and not args.no_cpu_baseline:
                for mode, x in (("f64", x64), ("mixed", xm), ("mixed16", xh)):
                    keep_solutions[f"{fmt}/{mode}"] = hrd.unpack_spinor(x, dims, fmt, "f64", "even").cpu().numpy() \
                        .reshape(psi_np.shape)
            # 4. fermion force from the mixed solution
            r[f"action_force_{fmt}_ms"], _ = rec.timed_once(f"action_force_{fmt}",
                                                            lambda: hrd.action_force(U64, xm, m0, dims, fmt))
            # 5. batched multi-RHS D^ (FP32)
            if batched_ok:
                srcs = torch.stack([hrd.convert_spinor(hrd.pack_spinor(t, dims, fmt, "f64", "even"), dims, fmt,
                                                       1, True) for t in rhs_nat])
                dsts = torch.empty_like(srcs)
                probs = hrd.make_problems([{"dims": dims, "rep": fmt, "nrhs": nrhs_batched, "m0": m0, "U32": U32,
                                            "src": srcs, "dst": dsts}])
                wb = torch.empty(max(hrd.batched_workspace_bytes(probs, "eo"), 1), dtype=torch.uint8, device=dev)
                L, S = _ls(fmt, "f32")
                r[f"batched_dhat_{fmt}"] = rec.timed(
                    f"batched_dhat_f32_{fmt}", lambda: hrd.dirac_apply_batched(probs, "eo", tune=tunes[fmt], work=wb),
                    5, 2, V * 8 * L + (V // 2) * 5 * S * nrhs_batched,
                    nrhs_batched * dhat_conv_bytes(V, fmt, "f32") - (nrhs_batched - 1) * V * 8 * L, V * nrhs_batched)
                del srcs, dsts, wb
            # 6. clover-improved operator (fundamental links only)
            if fmt == "fund":
                for kind in CLOVER_KINDS:
                    r[f"clover_build_{kind}_ms"], c64 = rec.timed_once(
                        f"clover_build_{kind}", lambda: hrd.clover_build(U64, CSW, m0, dims, fmt, kind=kind))
                    c32 = hrd.convert_clover(c64, dims, fmt)
                    cd64 = hrd.CloverOp(U64, c64, dims, fmt, "eo")
                    cd32 = hrd.CloverOp(U32, c32, dims, fmt, "eo")
                    for prec, cd in (("f64", cd64), ("f32", cd32)):
                        r[f"dhat_clover_{kind}_{prec}"] = rec.timed(
                            f"dhat_clover_{kind}_{prec}_fund", lambda: cd(lo[prec]["e"], outs[prec]["e"]), R // 2, 2,
                            dhat_clover_alg_bytes(V, "fund", prec), None, V)
                    r[f"cg_clover_{kind}_f64_ms"], (_, ic64) = rec.timed_once(
                        f"cg_clover_{kind}_f64",
                        lambda: hrd.cg_solve_clover(U64, c64, src_e, tol, dims, fmt, mode="f64"))
                    r[f"cg_clover_{kind}_mixed_ms"], (_, icm) = rec.timed_once(
                        f"cg_clover_{kind}_mixed",
                        lambda: hrd.cg_solve_clover(U64, c64, src_e, tol, dims, fmt, mode="mixed", U32=U32,
                                                    clov32=c32))
                    r[f"cg_clover_{kind}_mixed16_ms"], (_, ich) = rec.timed_once(
                        f"cg_clover_{kind}_mixed16",
                        lambda: hrd.cg_solve_clover(U64, c64, src_e, tol, dims, fmt, mode="mixed16", U32=U16,
                                                    clov32=c32))
                    r[f"cg_clover_{kind}_f64"], r[f"cg_clover_{kind}_mixed"] = ic64, icm
                    r[f"cg_clover_{kind}_mixed16"] = ich
                    del c64, c32, cd64, cd32
            del U64, U32, U16, Us, x64, xm, xh, d
        return r

    tunes = {}
    if batched_ok:
        # launch shape of the batched stages, chosen by the library's autotuner (untimed setup)
        for fmt in LINK_FORMATS:
            U32t = hrd.convert_gauge(hrd.pack_gauge(U_nat, dims, fmt, "f64"), dims, fmt)
            srcs = torch.zeros((nrhs_batched, hrd.spinor_bytes(dims, fmt, "f32", 1)), dtype=torch.uint8, device=dev)
            probs = hrd.make_problems([{"dims": dims, "rep": fmt, "nrhs": nrhs_batched, "m0": m0, "U32": U32t,
                                        "src": srcs, "dst": torch.zeros_like(srcs)}])
            tunes[fmt] = hrd.autotune_batched(probs, cache_path=args.tune_cache)
            print(f"[bench] batched tune {fmt}: {tunes[fmt]}", file=sys.stderr, flush=True)
            del U32t, srcs, probs
    for w in range(args.warmup):
        print(f"[bench] warmup {w}", file=sys.stderr, flush=True)
        step(False)
    rec.entries.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = []
    for s_ in range(args.steps):
        per.append(step(s_ == args.steps - 1))
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
        for kind in ("hop", "full", "dhat"):
            for prec in ("f64", "f32", "f16"):
                key = f"{kind}_{prec}_{fmt}"
                alg_f, conv_f, _, sf = OPS[kind]
                dslash[key] = dslash_entry(avg(key), alg_f(V, fmt, prec), conv_f(V, fmt, prec), int(V * sf))
                attach_measured(dslash[key], key, summ)
        key = f"dhat_dag_f64_{fmt}"
        dslash[key] = dslash_entry(avg(key), dhat_alg_bytes(V, fmt, "f64"), dhat_conv_bytes(V, fmt, "f64"), V)
        attach_measured(dslash[key], key, summ)
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
            attach_measured(d_[f"dhat_{prec}"], f"dhat_clover_{kind}_{prec}_fund", summ)
        d_["cg_f64"] = {"ms": avg(f"cg_clover_{kind}_f64_ms"), **per[-1][f"cg_clover_{kind}_f64"]}
        d_["cg_mixed"] = {"ms": avg(f"cg_clover_{kind}_mixed_ms"), **per[-1][f"cg_clover_{kind}_mixed"]}
        d_["cg_mixed16"] = {"ms": avg(f"cg_clover_{kind}_mixed16_ms"), **per[-1][f"cg_clover_{kind}_mixed16"]}
        d_["mixed_over_f64_time"] = d_["cg_mixed"]["ms"] / d_["cg_f64"]["ms"]
        d_["mixed16_over_f64_time"] = d_["cg_mixed16"]["ms"] / d_["cg_f64"]["ms"]
        clover[kind] = d_
    hop = dslash["hop_f64_fund"]
    hop_gbs = hop["alg_GBs"]
    roof = {"bound": "hbm", "achieved": round(hop_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(hop_gbs / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "hop_kernel<FUND, double, dagger=false, no epilogue>",
            "alg_bytes_per_launch": hop_alg_bytes(V, "fund", "f64"), "avg_launch_ms": hop["ms"],
            "timing": "HIP events around R back-to-back launches on the library's stream"}
    if "traffic_bytes" in hop:
        roof["traffic"] = hop["traffic_bytes"]
        roof["traffic_over_alg"] = hop["traffic_over_alg"]
        roof["traffic_source"] = ("rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs of this benchmark, calibrated "
                                  "on the stream probe's 1:1 copy of known size (profiles/"
                                  "bench_48x48x48x48_sections.md)")
    if "rocprof_ms" in hop:
        roof["rocprof_avg_launch_ms"] = hop["rocprof_ms"]
        roof["frac_at_rocprof_duration"] = round(hop["alg_GBs_at_rocprof_ms"] / HBM_PEAK_GBS, 4)
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
        "roofline": roof,
        "dslash": dslash,
        "cg": cg,
        "clover": clover,
        "library": hrd.version(),
        "profile_summary_matches_library": summ is not None,
    }
    if batched_ok:
        out["batched"] = {}
        for fmt in LINK_FORMATS:
            bms = avg(f"batched_dhat_{fmt}")
            L, S = _ls(fmt, "f32")
            bbytes = V * 8 * L + (V // 2) * 5 * S * nrhs_batched
            e = {"nrhs": nrhs_batched, "dhat_f32_ms": bms, "ms": bms, "alg_bytes": bbytes,
                 "alg_GBs": bbytes / (bms * 1e-3) / 1e9, "pct_hbm_peak": 100.0 * bbytes / (bms * 1e-3) / 1e9 /
                 HBM_PEAK_GBS, "ms_per_rhs": bms / nrhs_batched, "tune": tunes[fmt],
                 "single_dhat_f32_ms": avg(f"dhat_f32_{fmt}")}
            attach_measured(e, f"batched_dhat_f32_{fmt}", summ)
            out["batched"][fmt] = e
    print("[bench] stream-probe ceiling", file=sys.stderr, flush=True)
    out["ceiling"] = stream_ceiling(torch, hrd, rec, dev)
    for name in out["ceiling"]:
        attach_measured(out["ceiling"][name], name, summ)
    if not args.no_adj48:
        print("[bench] SU(2) adjoint at 48^4", file=sys.stderr, flush=True)
        out["adjoint48"] = adjoint48_stage(torch, hrd, inputs, rec, summ, U_nat, dims)
    if batched_ok and not args.no_config4:
        print("[bench] mixed-volume batched CG", file=sys.stderr, flush=True)
        out["batched_cg_mixed_volumes"] = mixed_volume_cg(torch, hrd, inputs, dev)
    if not args.no_sun:
        print("[bench] SU(2) adjoint stage", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_stage(torch, hrd, inputs, dev)
        print("[bench] SU(3) representations stage", file=sys.stderr, flush=True)
        out["sun"] = sun_stage(torch, hrd, inputs, dev)
        print("[bench] SU(4) representations stage", file=sys.stderr, flush=True)
        out["sun4"] = sun_stage(torch, hrd, inputs, dev, dims=(24, 24, 24, 24), nc=4)
    if args.manifest:
        with open(args.manifest, "w") as f:
            json.dump({"dims": list(dims), "library": hrd.version(), "source_hash": hrd.build_hash(),
                       "sections": rec.entries}, f)
    if not args.no_cpu_baseline:
        del U_nat, psi_nat
        torch.cuda.empty_cache()
        print("[bench] CPU oracle: hopping term", file=sys.stderr, flush=True)
        cb = cpu_oracle_baseline(U_np, psi_np, V)
        model, nproc, threads = cpu_info()
        cb.update({"cpu_model": model, "nproc": nproc, "omp_threads": threads})
        print("[bench] CPU oracle: configurations", file=sys.stderr, flush=True)
        cb["configs"] = cpu_oracle_configs(inputs, U_np, psi_np, m0, with_cg=not args.no_oracle_cg)
        if not args.no_oracle_cg and keep_solutions:
            import oracle as O

            print("[bench] CPU oracle: FP64 CG to 1e-12 at 48^4", file=sys.stderr, flush=True)
            cb["solution_error_48"] = oracle_solution_errors(U_np, O.restrict(psi_np, 0), m0, keep_solutions)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# profile summariser: rocprofv3 runs of this command -> profiles/*
# ---------------------------------------------------------------------------

def _read_csv(pattern_dir, suffix):
    files = sorted(glob.glob(os.path.join(pattern_dir, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {pattern_dir}")
    rows = []
    for fn in files:
        with open(fn, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _grid(row):
    if "Grid_Size" in row and row["Grid_Size"] not in (None, ""):
        return int(row["Grid_Size"])
    return int(row.get("Grid_Size_X", 1)) * int(row.get("Grid_Size_Y", 1)) * int(row.get("Grid_Size_Z", 1))


def _is_marker(name, grid):
    return "stream_probe_kernel" in name and grid <= 256


def _dispatches_trace(d):
    rows = _read_csv(d, "kernel_trace.csv")
    out = [{"id": int(r.get("Dispatch_Id") or r["Correlation_Id"]), "name": r["Kernel_Name"], "grid": _grid(r),
            "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])} for r in rows]
    return sorted(out, key=lambda x: x["id"])


def _dispatches_counters(d):
    rows = _read_csv(d, "counter_collection.csv")
    by = {}
    for r in rows:
        k = int(r["Dispatch_Id"])
        e = by.setdefault(k, {"id": k, "name": r["Kernel_Name"], "grid": _grid(r), "c": {}})
        e["c"][r["Counter_Name"]] = e["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [by[k] for k in sorted(by)]


def _split(disp, n_sections, what):
    marks = [i for i, x in enumerate(disp) if _is_marker(x["name"], x["grid"])]
    if len(marks) != 2 * n_sections:
        raise SystemExit(f"{what}: {len(marks)} marker dispatches for {n_sections} sections")
    return [disp[marks[2 * k] + 1:marks[2 * k + 1]] for k in range(n_sections)]


def _short(name):
    n = name.replace("hrd::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    n = n.replace("hrd::", "")
    if n.startswith("void "):
        n = n[5:]
    return n.split("(")[0] if "(" in n else n


def summarize(args):
    man = json.load(open(args.manifest))
    secs = man["sections"]
    ns = len(secs)
    res = {}
    commands = [c for c in (args.cmd or [])]
    if args.trace:
        segs = _split(_dispatches_trace(args.trace), ns, "kernel trace")
        for s, seg in zip(secs, segs):
            e = res.setdefault(s["name"], {"reps": 0, "ns": 0, "dispatches": 0, "kernels": {}})
            e["reps"] += s["reps"]
            e["ns"] += sum(x["ns"] for x in seg)
            e["dispatches"] += len(seg)
            for x in seg:
                k = e["kernels"].setdefault(_short(x["name"]), [0, 0])
                k[0] += 1
                k[1] += x["ns"]
    counters = {}
    for label, d in (("fetch", args.fetch), ("write", args.write), ("tcc", args.tcc), ("sq", args.sq)):
        if not d:
            continue
        segs = _split(_dispatches_counters(d), ns, label)
        for s, seg in zip(secs, segs):
            e = counters.setdefault(s["name"], {})
            for x in seg:
                for cn, cv in x["c"].items():
                    e.setdefault(cn, [0.0, 0])
                    e[cn][0] += cv
            for cn in e:
                pass
            e.setdefault("_reps_" + label, 0)
            e["_reps_" + label] += s["reps"]
    # calibration on the stream probe's copy (bytes known exactly)
    cal = None
    if "probe_copy" in counters and "FETCH_SIZE" in counters["probe_copy"] and "WRITE_SIZE" in counters["probe_copy"]:
        c = counters["probe_copy"]
        man_copy = next(s for s in secs if s["name"] == "probe_copy")
        half = man_copy["alg_bytes"] // 2  # the copy reads and writes the same number of bytes
        fk = c["FETCH_SIZE"][0] / c["_reps_fetch"] * 1024.0
        wk = c["WRITE_SIZE"][0] / c["_reps_write"] * 1024.0
        cal = {"copy_bytes_each_way": half, "fetch_factor": half / fk, "write_factor": half / wk}
    summary = {"source_hash": man["source_hash"], "library": man["library"], "dims": man["dims"],
               "calibration": cal, "commands": commands, "sections": {}}
    first = {}
    for s in secs:
        first.setdefault(s["name"], s)
    for name, s in first.items():
        out = {"reps_profiled": None, "rocprof_ms": None, "alg_bytes": s["alg_bytes"], "conv_bytes": s["conv_bytes"],
               "launches": s["launches"]}
        if name in res:
            e = res[name]
            out["reps_profiled"] = e["reps"]
            out["rocprof_ms"] = e["ns"] / e["reps"] / 1e6
            out["dispatches_per_app"] = e["dispatches"] / e["reps"]
            out["kernels"] = {k: {"dispatches": v[0], "avg_us": v[1] / v[0] / 1e3} for k, v in e["kernels"].items()}
        if name in counters:
            c = counters[name]
            if cal and "FETCH_SIZE" in c:
                out["read_bytes"] = c["FETCH_SIZE"][0] / c["_reps_fetch"] * 1024.0 * cal["fetch_factor"]
            if cal and "WRITE_SIZE" in c:
                out["write_bytes"] = c["WRITE_SIZE"][0] / c["_reps_write"] * 1024.0 * cal["write_factor"]
            if "read_bytes" in out and "write_bytes" in out:
                out["traffic_bytes"] = out["read_bytes"] + out["write_bytes"]
                if s["alg_bytes"]:
                    out["traffic_over_alg"] = out["traffic_bytes"] / s["alg_bytes"]
                if out["rocprof_ms"]:
                    out["dram_GBs_at_rocprof_ms"] = out["traffic_bytes"] / (out["rocprof_ms"] * 1e-3) / 1e9
            for cn in c:
                if cn.startswith("_") or cn in ("FETCH_SIZE", "WRITE_SIZE"):
                    continue
                reps = c.get("_reps_tcc") if cn.startswith("TCC") else c.get("_reps_sq")
                if reps:
                    out.setdefault("counters_per_app", {})[cn] = c[cn][0] / reps
        if out["rocprof_ms"] and s["alg_bytes"]:
            out["alg_GBs_at_rocprof_ms"] = s["alg_bytes"] / (out["rocprof_ms"] * 1e-3) / 1e9
            out["alg_pct_hbm_peak_at_rocprof_ms"] = 100.0 * out["alg_GBs_at_rocprof_ms"] / HBM_PEAK_GBS
        summary["sections"][name] = out
    with open(args.out + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    lines = [f"# Timed sections of the benchmark at {'x'.join(map(str, man['dims']))} under rocprofv3", "",
             f"Library: `{man['library']}` (source hash `{man['source_hash']}`).", "", "Commands:", "", "```"]
    lines += commands + ["```", ""]
    if cal:
        lines += [f"Calibration: the stream probe's copy moves {cal['copy_bytes_each_way']} bytes each way; its "
                  f"FETCH_SIZE gives x{cal['fetch_factor']:.3f} and its WRITE_SIZE x{cal['write_factor']:.3f} "
                  f"(factors applied to every section).", ""]
    lines += ["Per application of each section: rocprof duration (sum of its kernels' durations / repetitions), "
              "algorithmic bytes and their rate at that duration, calibrated HBM bytes (FETCH_SIZE + WRITE_SIZE) "
              "and their ratio to the algorithmic bytes, and the DRAM rate at the rocprof duration.", "",
              "| section | rocprof ms | alg GB | alg GB/s | % of 8 TB/s | HBM GB | HBM/alg | DRAM GB/s | "
              "L2 hit % |", "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]

    def f_(v, fmt):
        return "" if v is None else format(v, fmt)

    for name, o in summary["sections"].items():
        cpa = o.get("counters_per_app", {})
        hit, miss = cpa.get("TCC_HIT_sum"), cpa.get("TCC_MISS_sum")
        hr = 100.0 * hit / (hit + miss) if hit is not None and miss is not None and hit + miss > 0 else None
        lines.append(f"| {name} | {f_(o['rocprof_ms'], '.4f')} | {f_(o['alg_bytes'] and o['alg_bytes'] / 1e9, '.4f')}"
                     f" | {f_(o.get('alg_GBs_at_rocprof_ms'), '.0f')} | "
                     f"{f_(o.get('alg_pct_hbm_peak_at_rocprof_ms'), '.1f')} | "
                     f"{f_(o.get('traffic_bytes') and o['traffic_bytes'] / 1e9, '.4f')} | "
                     f"{f_(o.get('traffic_over_alg'), '.3f')} | {f_(o.get('dram_GBs_at_rocprof_ms'), '.0f')} | "
                     f"{f_(hr, '.1f')} |")
    lines += ["", "Kernels per section (dispatches, average duration under the profiler):", ""]
    for name, o in summary["sections"].items():
        if "kernels" in o:
            ks = "; ".join(f"`{k}` x{v['dispatches']} {v['avg_us']:.1f} us" for k, v in o["kernels"].items())
            lines.append(f"* {name}: {ks}")
    sq = [(n, o["counters_per_app"]) for n, o in summary["sections"].items()
          if any(k.startswith("SQ") or k.startswith("GRBM") for k in o.get("counters_per_app", {}))]
    if sq:
        names = sorted({k for _, c in sq for k in c if k.startswith("SQ") or k.startswith("GRBM")})
        lines += ["", "Shader counters per application:", "", "| section | " + " | ".join(names) + " |",
                  "|---|" + "---:|" * len(names)]
        for n, c in sq:
            lines.append(f"| {n} | " + " | ".join(f_(c.get(k), ".4g") for k in names) + " |")
    with open(args.out + ".md", "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {args.out}.json and {args.out}.md ({len(summary['sections'])} sections)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--reps", type=int, default=50, help="Dslash applications timed per step")
    ap.add_argument("--dims", type=str, default="48,48,48,48")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-cg", action="store_true", help="skip the oracle CG solves on the CPU")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-adj48", action="store_true", help="skip the 48^4 adjoint sections")
    ap.add_argument("--no-config4", action="store_true", help="skip the mixed-volume batched CG comparison")
    ap.add_argument("--no-sun", action="store_true", help="skip the 32^4 adjoint and SU(3) stages")
    ap.add_argument("--tune-cache", type=str, default=None, help="JSON-lines cache file of the batched autotuner")
    ap.add_argument("--manifest", type=str, default=None, help="write the list of timed sections to this file")
    ap.add_argument("--summarize", action="store_true",
                    help="summarise rocprofv3 runs of this command (--manifest, --trace, --fetch, ...)")
    ap.add_argument("--trace", type=str, default=None, help="rocprofv3 --kernel-trace output directory")
    ap.add_argument("--fetch", type=str, default=None, help="rocprofv3 --pmc FETCH_SIZE output directory")
    ap.add_argument("--write", type=str, default=None, help="rocprofv3 --pmc WRITE_SIZE output directory")
    ap.add_argument("--tcc", type=str, default=None, help="rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum output directory")
    ap.add_argument("--sq", type=str, default=None, help="rocprofv3 --pmc run of SQ/GRBM counters")
    ap.add_argument("--cmd", action="append", help="command line recorded in the summary (repeatable)")
    ap.add_argument("--out", type=str, default=os.path.join(ROOT, "profiles", "bench_48x48x48x48_sections"))
    args = ap.parse_args()
    if args.summarize:
        summarize(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the lattice is not sharded "
                                   "across GPUs (see the design notes on sharding)", "n_gpus": args.gpus}))
        sys.exit(2)
    run(args)


if __name__ == "__main__":
    main()
