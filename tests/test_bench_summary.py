"""Host logic of the benchmark's profile summariser (no GPU): a synthetic
rocprofv3 kernel trace and counter collection of a run with three timed
sections are split at the marker dispatches and reduced to per-application
durations, calibrated HBM bytes and L2 hit counts."""
import csv
import json
import os
import sys
from types import SimpleNamespace

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

MARK = "void hrd::(anonymous namespace)::stream_probe_kernel<0>(double2 const*, double2*, long, int)"
HOP = "void hrd::(anonymous namespace)::hop_kernel<0, double, false, false, false, false, false, 0>(hrd::HopArgs)"
PROBE = "void hrd::(anonymous namespace)::stream_probe_kernel<0>(double2 const*, double2*, long, int)"


def _run(tmp_path):
    # sections: probe_copy (2 reps, 1 GiB each way), hop (3 reps), dhat (1 rep, two launches)
    seq = [("setup", 1 << 20, 5000)]
    seq += [("mark", 256, 10)] + [("probe", 1 << 26, 400_000)] * 2 + [("mark", 256, 10)]
    seq += [("mark", 256, 10)] + [("hop", 2654208, 390_000)] * 3 + [("mark", 256, 10)]
    seq += [("mark", 256, 10)] + [("hop", 2654208, 380_000), ("hop", 2654208, 400_000)] + [("mark", 256, 10)]
    names = {"mark": MARK, "probe": PROBE, "hop": HOP, "setup": "void other_kernel()"}
    tr = tmp_path / "trace"
    tr.mkdir()
    with open(tr / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X",
                    "Grid_Size_Y", "Grid_Size_Z"])
        t = 1000
        for i, (k, g, ns) in enumerate(seq):
            w.writerow(["KERNEL_DISPATCH", i + 1, names[k], t, t + ns, g, 1, 1])
            t += ns + 100
    counters = {"fetch": {"probe": {"FETCH_SIZE": 524288.0}, "hop": {"FETCH_SIZE": 945000.0}},
                "write": {"probe": {"WRITE_SIZE": 1048576.0}, "hop": {"WRITE_SIZE": 331776.0}},
                "tcc": {"probe": {"TCC_HIT_sum": 0.0, "TCC_MISS_sum": 1.0},
                        "hop": {"TCC_HIT_sum": 18.0e6, "TCC_MISS_sum": 17.0e6}}}
    for label, per in counters.items():
        d = tmp_path / label
        d.mkdir()
        with open(d / "run_counter_collection.csv", "w", newline="") as f:
            w = csv.writer(f)
            w.writerow(["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"])
            for i, (k, g, _) in enumerate(seq):
                for cn, cv in per.get(k, {"FETCH_SIZE" if label == "fetch" else
                                          "WRITE_SIZE" if label == "write" else "TCC_HIT_sum": 1.0}).items():
                    w.writerow([i + 1, g, names[k], cn, cv])
    man = {"dims": [48, 48, 48, 48], "library": "hrd test", "source_hash": "0123456789abcdef",
           "sections": [{"name": "probe_copy", "reps": 2, "launches": 1, "alg_bytes": 2 << 30, "conv_bytes": 2 << 30,
                         "sites": None, "ms": 0.4},
                        {"name": "hop_f64_fund", "reps": 3, "launches": 1, "alg_bytes": 2038431744,
                         "conv_bytes": None, "sites": 2654208, "ms": 0.39},
                        {"name": "dhat_f64_fund", "reps": 1, "launches": 2, "alg_bytes": 4416602112,
                         "conv_bytes": None, "sites": 5308416, "ms": 0.79}]}
    mp = tmp_path / "manifest.json"
    mp.write_text(json.dumps(man))
    out = tmp_path / "summary"
    args = SimpleNamespace(manifest=str(mp), trace=str(tr), fetch=str(tmp_path / "fetch"),
                           write=str(tmp_path / "write"), tcc=str(tmp_path / "tcc"), sq=None, cmd=["cmd a"],
                           out=str(out))
    bench.summarize(args)
    return json.loads((tmp_path / "summary.json").read_text()), (tmp_path / "summary.md").read_text()


def test_sections_are_split_at_the_markers(tmp_path):
    s, md = _run(tmp_path)
    sec = s["sections"]
    assert abs(sec["hop_f64_fund"]["rocprof_ms"] - 0.39) < 1e-12
    assert abs(sec["dhat_f64_fund"]["rocprof_ms"] - 0.78) < 1e-12
    assert sec["dhat_f64_fund"]["dispatches_per_app"] == 2
    assert abs(sec["probe_copy"]["rocprof_ms"] - 0.4) < 1e-12
    assert "hop_f64_fund" in md and "cmd a" in md


def test_counters_are_calibrated_on_the_copy(tmp_path):
    s, _ = _run(tmp_path)
    cal = s["calibration"]
    # the copy moves 1 GiB each way; FETCH_SIZE reported 0.5 GiB, WRITE_SIZE 1 GiB
    assert abs(cal["fetch_factor"] - 2.0) < 1e-12 and abs(cal["write_factor"] - 1.0) < 1e-12
    hop = s["sections"]["hop_f64_fund"]
    assert abs(hop["read_bytes"] - 945000.0 * 1024 * 2) < 1e-3
    assert abs(hop["write_bytes"] - 331776.0 * 1024) < 1e-3
    assert abs(hop["traffic_over_alg"] - (945000.0 * 2048 + 331776.0 * 1024) / 2038431744) < 1e-12
    assert abs(hop["counters_per_app"]["TCC_HIT_sum"] - 18.0e6) < 1e-6
