"""Profiling helpers for the evaluator kernels (run under rocprofv3).

  python -m paper_2603_12292_amd.profiling run [--steps N] [--adjoint]
      one warm-up and N evaluations of the benchmark workload (plain-mid,
      correlation fitness; --adjoint: fitness and constant gradients of the
      differentiation workload, MSE), then a 256 MiB device-to-device copy whose byte
      count is known, used to scale the HBM counters.

  python -m paper_2603_12292_amd.profiling summarize --trace DIR --fetch CSV --write CSV [--valu CSV] --out PREFIX
      reads the rocprofv3 kernel-trace statistics and the FETCH_SIZE /
      WRITE_SIZE counter CSVs of the run above and writes
      PREFIX.txt (duration and traffic summary) and PREFIX_traffic.json
      (HBM bytes per launch of the interpreter kernel, with the hash of the
      kernel sources the counters were taken on).

FETCH_SIZE and WRITE_SIZE count KiB moved between L2 and memory per
dispatch; each is scaled by (known bytes / counted bytes) of the calibration
copy, which reads and writes exactly COPY_BYTES.  SQ_INSTS_VALU (wave-level
VALU instructions per dispatch) times 64 lanes over the traced average
duration gives the VALU lane-operations issued per second, against the
chip's 39.3 T lane-operations/s (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 256 << 20
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# the correlation-fitness interpreter of the common register-need class; its
# tile-width variant (<1, 0, 0>: 8 cases per lane, <1, 0, 1>: 4) is the one
# the tuner picked, i.e. the one with the largest total time in the trace
KERNEL_PREFIX = "k_eval_class<1, 0, "
EVAL_SOURCES = ["eval.hip", "beagle_device.h", "kernels.h", "trig.h"]


def source_hash() -> str:
    h = hashlib.sha256()
    for f in EVAL_SOURCES:
        with open(os.path.join(ROOT, "paper_2603_12292_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def run(steps: int, adjoint: bool = False):
    import torch
    sys.path.insert(0, ROOT)
    from paper_2603_12292_amd import api
    from paper_2603_12292_amd import workloads as wl
    w = wl.config_differentiation() if adjoint else wl.config_mid()
    progs = api.DevicePrograms.from_programset(w.programs, "cuda:0")
    X = torch.from_numpy(w.data.X).cuda()
    y = torch.from_numpy(w.data.y).cuda()
    call = (lambda: api.evaluate_grad(progs, X, y, "mse")) if adjoint else (lambda: api.evaluate(progs, X, y, "corr"))
    call()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"profiled {steps} evaluation(s) of {w.name} and a {COPY_BYTES} byte copy", flush=True)


def _counter_rows(path):
    per = defaultdict(dict)
    names = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            per[d][r["Counter_Name"]] = float(r["Counter_Value"])
            names[d] = r["Kernel_Name"]
    return per, names


def _counter(path, counter, kernel):
    per, names = _counter_rows(path)
    evals = [per[d][counter] for d in sorted(per) if kernel in names[d]]
    copies = [per[d][counter] for d in sorted(per)
              if "k_eval" not in names[d] and ("copy" in names[d].lower() or "elementwise" in names[d].lower())]
    return evals, copies


def summarize(trace_dir, fetch_csv, write_csv, out_prefix, command, valu_csv=None):
    stats = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    lines = []
    kern_ms = None
    kernel = None
    if stats:
        with open(stats[0]) as f:
            rows = list(csv.DictReader(f))
        rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
        lines.append("kernel-trace statistics (ns):")
        lines.append(f"{'calls':>6} {'average':>12} {'total':>14} {'%':>6}  name")
        for r in rows[:12]:
            lines.append(f"{int(r['Calls']):6d} {float(r['AverageNs']):12.1f} {float(r['TotalDurationNs']):14.1f} "
                         f"{float(r['Percentage']):6.2f}  {r['Name'][:90]}")
            if kernel is None and KERNEL_PREFIX in r["Name"]:
                kernel = r["Name"][r["Name"].index("k_eval_class"):r["Name"].index(">") + 1]
                kern_ms = float(r["AverageNs"]) / 1e6
    rec = {"kernel": kernel, "source_hash": source_hash(), "avg_ms": kern_ms}
    if fetch_csv and write_csv and kernel:
        fe, fc = _counter(fetch_csv, "FETCH_SIZE", kernel)
        we, wc = _counter(write_csv, "WRITE_SIZE", kernel)
        f_scale = COPY_BYTES / (max(fc) * 1024) if fc else None
        w_scale = COPY_BYTES / (max(wc) * 1024) if wc else None
        fetch = fe[-1] * 1024 * f_scale if fe and f_scale else None
        write = we[-1] * 1024 * w_scale if we and w_scale else None
        rec.update({"fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
                    "fetch_scale": f_scale, "write_scale": w_scale,
                    "hbm_bytes_per_launch": (fetch + write) if fetch is not None and write is not None else None})
        lines.append("")
        lines.append("HBM traffic of one interpreter launch (FETCH_SIZE / WRITE_SIZE, KiB counters scaled by a")
        lines.append(f"{COPY_BYTES} byte copy: fetch x{f_scale:.4f}, write x{w_scale:.4f}):" if f_scale and w_scale
                     else "HBM traffic: calibration copy not found")
        if fetch is not None and write is not None:
            lines.append(f"  fetch {fetch / 1e6:.3f} MB  write {write / 1e6:.3f} MB  total {(fetch + write) / 1e6:.3f} MB")
    if valu_csv and kernel and kern_ms:
        ve, _ = _counter(valu_csv, "SQ_INSTS_VALU", kernel)
        if ve:
            lane_ops = ve[-1] * 64
            rate = lane_ops / (kern_ms * 1e-3)
            rec.update({"valu_lane_ops_per_launch": lane_ops, "valu_lane_ops_per_s": rate,
                        "valu_issue_frac": rate / PEAK_LANE_OPS})
            lines.append("")
            lines.append(f"VALU issue (SQ_INSTS_VALU x 64 / traced average duration): {lane_ops:.4g} lane-ops per launch, "
                         f"{rate / 1e12:.2f} T lane-ops/s = {rate / PEAK_LANE_OPS:.3f} of {PEAK_LANE_OPS / 1e12:.1f} T")
    lines.insert(0, f"command: {command}")
    lines.insert(1, f"kernel {kernel}, source hash {rec['source_hash']}")
    with open(out_prefix + ".txt", "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(out_prefix + "_traffic.json", "w") as f:
        json.dump(rec, f, indent=1)
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--steps", type=int, default=1)
    r.add_argument("--adjoint", action="store_true",
                   help="fitness and constant gradients of the differentiation workload instead")
    s = sub.add_parser("summarize")
    s.add_argument("--trace", required=True)
    s.add_argument("--fetch")
    s.add_argument("--write")
    s.add_argument("--valu")
    s.add_argument("--out", required=True)
    s.add_argument("--command", default="")
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.steps, a.adjoint)
    else:
        summarize(a.trace, a.fetch, a.write, a.out, a.command, a.valu)


if __name__ == "__main__":
    main()
