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

  python -m paper_2603_12292_amd.profiling ops
      one evaluation per single-operator program shape (see OP_SHAPES), each
      a population of 1024 identical programs on 2^17 cases, MSE, 4 cases
      per lane: run under rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU.

  python -m paper_2603_12292_amd.profiling paper [--steps N] [--kind mse]
      one warm-up and N evaluations of the paper-regime population (2^20
      programs on 512 cases).

  python -m paper_2603_12292_amd.profiling summarize-kernels --trace DIR --pmc DIR... --kernels a,b --out PREFIX
      per named kernel: kernel-trace duration and the mean per dispatch of
      every counter of the given counter runs (PREFIX.txt, PREFIX.json).

  python -m paper_2603_12292_amd.profiling summarize-ops --pmc CSV --out PREFIX
      per-operator VALU lane-operations and SALU instructions per node-case
      from that run (PREFIX.txt).

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


# Single-operator program shapes (D = 1, x0 in [1, 2]).  Every shape's cost
# above the one-token program "x0" is divided by its count of the measured
# unit: a unary operator; a "push x0, binary operator" pair whose right
# operand is a square root (its cost subtracted; the pair is not fused); a
# fused word "binary operator with a variable or constant operand" (two
# nodes, one decoded word).
OPS_N = 1024
OPS_M = 1 << 17
UNARY_NAMES = ("sin", "cos", "exp", "log", "sqrt")
BINARY_NAMES = ("+", "-", "*", "/")


def op_shapes():
    """[(name, tokens, consts, units, subtract)]; subtract: (shape, count)
    whose per-unit cost is removed first, or None."""
    from paper_2603_12292_amd import workloads as wl
    V, C = wl.tok(wl.VAR, 0), wl.tok(wl.CONST, 0)
    un = dict(zip(UNARY_NAMES, (wl.SIN, wl.COS, wl.EXP, wl.LOG, wl.SQRT)))
    bi = dict(zip(BINARY_NAMES, (wl.ADD, wl.SUB, wl.MUL, wl.DIV)))
    out = [("x0 (base)", [V], [], 0, None)]
    for n, op in un.items():
        out.append((n, [V] + [wl.tok(op)] * 63, [], 63, None))
    for n, op in bi.items():
        # x0 (x0 sqrt b)^21: 21 pushes, 21 square roots, 21 unfused binaries
        out.append((f"push+{n}", [V] + [V, wl.tok(wl.SQRT), wl.tok(op)] * 21, [], 21, ("sqrt", 21)))
        out.append((f"fused x0 {n}", [V] + [V, wl.tok(op)] * 31, [], 31, None))
        out.append((f"fused c0 {n}", [V] + [C, wl.tok(op)] * 31, [0.75], 31, None))
    return out


def run_ops():
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    from paper_2603_12292_amd import api
    from paper_2603_12292_amd import workloads as wl
    rng = np.random.default_rng(5)
    X = torch.from_numpy(rng.uniform(1.0, 2.0, (OPS_M, 1)).astype(np.float32)).cuda()
    y = torch.from_numpy(rng.uniform(0.0, 1.0, OPS_M).astype(np.float32)).cuda()
    ctx = api.Context(0)
    ctx.set_tuning("narrow")
    for name, toks, consts, _, _ in op_shapes():
        ps = wl.pack_programs([(toks, consts)] * OPS_N)
        api.evaluate(api.DevicePrograms.from_programset(ps, "cuda:0"), X, y, "mse", ctx=ctx)
        torch.cuda.synchronize()
        print(f"evaluated shape {name!r}", flush=True)
    ctx.close()


def summarize_ops(pmc_csv, out_prefix, command):
    per, names = _counter_rows(pmc_csv)
    # each evaluation launches one interpreter kernel per register-need
    # class; every shape here is class 0 at 4 cases per lane
    evals = [d for d in sorted(per) if "k_eval_class<0, 0, 1>" in names[d]]
    shapes = op_shapes()
    assert len(evals) == len(shapes), (len(evals), len(shapes))
    row = {s[0]: per[d] for s, d in zip(shapes, evals)}
    base = row["x0 (base)"]
    cases = OPS_N * OPS_M
    res = {}
    for name, toks, _, units, sub in shapes:
        if units == 0:
            continue
        v = (row[name]["SQ_INSTS_VALU"] - base["SQ_INSTS_VALU"]) * 64 / cases
        sa = (row[name]["SQ_INSTS_SALU"] - base["SQ_INSTS_SALU"]) * 64 / cases
        if sub:
            v -= res[sub[0]][0] * sub[1]
            sa -= res[sub[0]][1] * sub[1]
        res[name] = (v / units, sa / units)
    lines = [f"command: {command}",
             f"kernel k_eval_class<0, 0, 1> (MSE, register need <= 4, 4 cases per lane), source hash {source_hash()}",
             f"{OPS_N} identical programs per shape, D = 1, M = {OPS_M}, x0 ~ U(1, 2); cost above the program x0",
             "per unit and case: SQ_INSTS_VALU x 64 (VALU lane-operations) and SQ_INSTS_SALU x 64 (scalar",
             "instructions per 64 cases).  Units: a unary operator; push+b = pushing x0 and an unfused binary b",
             "(right operand a square root, its cost subtracted); fused = one decoded word, two nodes.",
             "",
             f"{'unit':<14} {'VALU lane-ops':>14} {'SALU x64':>10}"]
    for name, (v, sa) in res.items():
        lines.append(f"{name:<14} {v:14.2f} {sa:10.2f}")
    with open(out_prefix + ".txt", "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter_csv(path):
    """The counter CSV of a rocprofv3 run: `path` itself, or the one file
    named *counter_collection.csv below it."""
    if os.path.isdir(path):
        found = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
        if len(found) != 1:
            raise FileNotFoundError(f"expected one counter_collection.csv below {path}, found {found}")
        return found[0]
    return path


def _counter_rows(path):
    per = defaultdict(dict)
    names = {}
    with open(_counter_csv(path)) as f:
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
        se, _ = _counter(valu_csv, "SQ_INSTS_SALU", kernel)
        if ve:
            lane_ops = ve[-1] * 64
            rate = lane_ops / (kern_ms * 1e-3)
            rec.update({"valu_insts_per_launch": ve[-1], "valu_lane_ops_per_launch": lane_ops,
                        "valu_lane_ops_per_s": rate, "valu_issue_frac": rate / PEAK_LANE_OPS})
            lines.append("")
            lines.append(f"VALU issue (SQ_INSTS_VALU x 64 / traced average duration): {lane_ops:.4g} lane-ops per launch, "
                         f"{rate / 1e12:.2f} T lane-ops/s = {rate / PEAK_LANE_OPS:.3f} of {PEAK_LANE_OPS / 1e12:.1f} T")
        if se:
            rec["salu_insts_per_launch"] = se[-1]
            lines.append(f"SALU instructions per launch (SQ_INSTS_SALU): {se[-1]:.4g}")
    lines.insert(0, f"command: {command}")
    lines.insert(1, f"kernel {kernel}, source hash {rec['source_hash']}")
    with open(out_prefix + ".txt", "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(out_prefix + "_traffic.json", "w") as f:
        json.dump(rec, f, indent=1)
    print("\n".join(lines))


def run_paper(steps: int, kind: str = "mse"):
    """The paper-regime evaluation: 2^20 programs (plain-mid replicated 256
    times) on 512 cases, one warm-up and `steps` whole-population
    evaluations."""
    import torch
    sys.path.insert(0, ROOT)
    from paper_2603_12292_amd import api
    from paper_2603_12292_amd import workloads as wl
    w = wl.config_paper_shape()
    progs = api.DevicePrograms.from_programset(w.programs, "cuda:0")
    X = torch.from_numpy(w.data.X).cuda()
    y = torch.from_numpy(w.data.y).cuda()
    for _ in range(steps + 1):
        api.evaluate(progs, X, y, kind)
    torch.cuda.synchronize()
    print(f"profiled {steps} evaluation(s) of {w.name}, {kind}", flush=True)


def run_loop(generations: int, population: int = 5_000_000):
    """The paper's loop at its largest population: a ramped half-and-half
    population (depths 2..5, at most 64 tokens, the nine base operators) of
    `population` individuals, then `generations` rounds of correlation
    fitness on the paper-shape case set (512 cases, D = 5), microcosm
    selection (sample 100, keep 0.5) and mutation-only variation at the same
    size; one untimed round first."""
    import torch
    sys.path.insert(0, ROOT)
    from paper_2603_12292_amd import api
    from paper_2603_12292_amd import workloads as wl
    data = wl.config_paper_shape().data
    X = torch.from_numpy(data.X).cuda()
    y = torch.from_numpy(data.y).cuda()
    params = api.GenParams(tournament=1, p_crossover=0.0, p_mutation=1.0, max_len=64, max_consts=8,
                           init_depth_min=2, init_depth_max=5)
    ctx = api.context(0)
    pop = api.init_population(population, data.D, params, 2612, ctx=ctx)
    for g in range(generations + 1):
        fit = api.evaluate(pop.programs(), X, y, "corr", ctx=ctx)
        pop = api.generation_microcosm(pop.programs(), fit, params, data.D, 2612, g + 1, population,
                                       sample=100, keep=0.5, ctx=ctx)
    torch.cuda.synchronize()
    print(f"profiled {generations} generation(s) of the paper loop at {population} individuals", flush=True)


def run_ragged(steps: int):
    """The 64-problem ragged workload: one warm-up and `steps` batched
    evaluations (MSE, one replayed graph), then the same problems one call
    each."""
    import torch
    sys.path.insert(0, ROOT)
    from paper_2603_12292_amd import api
    from paper_2603_12292_amd import workloads as wl
    ws = wl.ragged_problems()
    dev = [(api.DevicePrograms.from_programset(w.programs, "cuda:0"), torch.from_numpy(w.data.X).cuda(),
            torch.from_numpy(w.data.y).cuda()) for w in ws]
    out = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p, _, _ in dev]
    ctx = api.context(0)
    for _ in range(steps + 1):
        api.evaluate_batched(dev, "mse", out=out, ctx=ctx)
    torch.cuda.synchronize()
    for p, X, y in dev:
        api.evaluate(p, X, y, "mse", ctx=ctx)
    torch.cuda.synchronize()
    print(f"profiled {steps} batched evaluation(s) of the ragged workload and one sequential pass", flush=True)


def summarize_kernels(trace_dir, pmc_dirs, kernels, out_prefix, command, title):
    """Per kernel whose name contains one of `kernels`: calls and average
    duration from the kernel trace, and the mean per dispatch of every
    counter of the counter runs."""
    stats = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    rows = []
    if stats:
        with open(stats[0]) as f:
            rows = list(csv.DictReader(f))
    lines = [f"command: {command}", title, "", "kernel-trace statistics (ns):",
             f"{'calls':>6} {'average':>12} {'total':>14} {'%':>6}  name"]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows[:16]:
        lines.append(f"{int(r['Calls']):6d} {float(r['AverageNs']):12.1f} {float(r['TotalDurationNs']):14.1f} "
                     f"{float(r['Percentage']):6.2f}  {r['Name'][:90]}")
    rec = {}
    for d in pmc_dirs:
        per, names = _counter_rows(d)
        for disp in sorted(per):
            for k in kernels:
                if k in names[disp]:
                    name = names[disp][:names[disp].find("(")] if "(" in names[disp] else names[disp]
                    slot = rec.setdefault(name, defaultdict(list))
                    for c, v in per[disp].items():
                        slot[c].append(v)
    lines += ["", "counters, mean per dispatch:"]
    summary = {}
    for name, cs in sorted(rec.items()):
        lines.append(f"  {name}")
        summary[name] = {}
        for c in sorted(cs):
            v = sum(cs[c]) / len(cs[c])
            summary[name][c] = v
            lines.append(f"    {c:<22} {v:16.6g}   ({len(cs[c])} dispatches)")
        w = summary[name].get("SQ_WAVES")
        for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM", "SQ_WAVE_CYCLES"):
            if w and c in summary[name]:
                lines.append(f"    {c + ' per wave':<34} {summary[name][c] / w:10.1f}")
    with open(out_prefix + ".txt", "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(out_prefix + ".json", "w") as f:
        json.dump(summary, f, indent=1)
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
    sub.add_parser("ops")
    lp = sub.add_parser("loop")
    lp.add_argument("--generations", type=int, default=3)
    rg = sub.add_parser("ragged")
    rg.add_argument("--steps", type=int, default=2)
    pp = sub.add_parser("paper")
    pp.add_argument("--steps", type=int, default=2)
    pp.add_argument("--kind", default="mse")
    sk = sub.add_parser("summarize-kernels")
    sk.add_argument("--trace", required=True)
    sk.add_argument("--pmc", nargs="*", default=[])
    sk.add_argument("--kernels", required=True, help="comma-separated name fragments")
    sk.add_argument("--out", required=True)
    sk.add_argument("--command", default="")
    sk.add_argument("--title", default="")
    so = sub.add_parser("summarize-ops")
    so.add_argument("--pmc", required=True)
    so.add_argument("--out", required=True)
    so.add_argument("--command", default="")
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.steps, a.adjoint)
    elif a.cmd == "ops":
        run_ops()
    elif a.cmd == "paper":
        run_paper(a.steps, a.kind)
    elif a.cmd == "ragged":
        run_ragged(a.steps)
    elif a.cmd == "loop":
        run_loop(a.generations)
    elif a.cmd == "summarize-kernels":
        summarize_kernels(a.trace, a.pmc, a.kernels.split(","), a.out, a.command, a.title)
    elif a.cmd == "summarize-ops":
        summarize_ops(a.pmc, a.out, a.command)
    else:
        summarize(a.trace, a.fetch, a.write, a.out, a.command, a.valu)


if __name__ == "__main__":
    main()
