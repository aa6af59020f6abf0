"""Benchmark of the population evaluator on one MI355X.

One step = one beagle_eval call on the plain-mid workload: N = 4096 postfix
programs (lengths uniform 5..64, up to 8 constants, op set + - * / sin cos exp
log sqrt), D = 5, M = 100000 fitness cases, correlation fitness 1 - r^2 with
binary64 sums.  Inputs are resident on the GPU before timing starts.  A step
covers program validation and decoding, case staging, the interpreter, the
per-case fitness terms, the reductions and the finalize.

Prints one JSON line:
  value          GPop/s = (sum of program lengths) * M * steps / seconds / 1e9
  roofline       the interpreter kernel against the chip's fp32 VALU lane
                 rate (see the roofline note below), with its duration
                 measured by HIP events on the kernel's stream
  cpu_baseline   the float64 CPU oracle on a bounded sample of the same
                 workload, on this host's cores
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# fp32 VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = one
# non-packed fp32 lane operation per lane per clock (the 157.3 TFLOP/s figure
# counts a packed two-wide FMA as 4 flops; a stack interpreter issues neither).
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
HBM_PEAK = 8.0e12


def function_nodes(ps) -> int:
    ops = ps.tokens & 0xFF
    return int(np.count_nonzero(ops < 9))


def committed_counters(kernel: str) -> dict:
    """Counter figures of the interpreter kernel from the committed profile
    summary (HBM bytes per launch, VALU issue fraction), or {} when the kernel
    source changed since they were taken or they are of another tile-width
    variant."""
    from paper_2603_12292_amd.profiling import source_hash
    path = os.path.join(ROOT, "profiles", "k_eval_class_corr_plain_mid_traffic.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash() or rec.get("kernel") != kernel:
        return {}
    return rec


def cpu_baseline(w, kind_id, budget_programs: int):
    from oracle import population as opop
    ps = w.programs
    # the pool's processes (one when the GPU runtime already runs: no fork then)
    cores = 1 if opop._gpu_runtime_started() else min(16, len(os.sched_getaffinity(0)))
    step = max(1, ps.n // budget_programs)
    sub = list(range(0, ps.n, step))[:budget_programs]
    nodes = int(ps.tok_len[sub].astype(np.int64).sum())
    t0 = time.perf_counter()
    opop.evaluate_population(ps.tokens, ps.tok_offset, ps.tok_len, ps.consts, ps.const_offset, ps.const_count,
                             w.data.X, w.data.y, kind_id, "o64", subset=sub, processes=cores)
    dt = time.perf_counter() - t0
    return {"value": nodes * w.data.M / dt / 1e9, "unit": "GPop/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sub)} of {ps.n} programs (every {step}), all {w.data.M} cases, "
                      f"correlation fitness, float64 oracle, {dt:.1f} s wall"}


def adjoint_bench(steps: int, warmup: int):
    """fwd+adjoint GPop/s on the differentiation workload (N=4096, 1..8
    constants, L~U{8..64}, D=5, M=100000), beside the plain evaluation of
    the same population, for the MSE and the correlation fitness (whose
    adjoint runs the evaluation first for its seeds); GPop/s counts each
    program node once per case."""
    import torch
    from paper_2603_12292_amd import api
    from paper_2603_12292_amd import workloads as wl
    w = wl.config_differentiation()
    progs = api.DevicePrograms.from_programset(w.programs, "cuda:0")
    X = torch.from_numpy(w.data.X).cuda()
    y = torch.from_numpy(w.data.y).cuda()
    nc = w.programs.node_count() * w.data.M

    def rate(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return nc * steps / (time.perf_counter() - t0) / 1e9

    fwd = rate(lambda: api.evaluate(progs, X, y, "mse"))
    both = rate(lambda: api.evaluate_grad(progs, X, y, "mse"))
    fwd_c = rate(lambda: api.evaluate(progs, X, y, "corr"))
    both_c = rate(lambda: api.evaluate_grad(progs, X, y, "corr"))
    # 20 Adam steps on every program's constants, end to end (adjoint,
    # optimizer update, final evaluation)
    from paper_2603_12292_amd import autograd as ag
    ag.tune_constants(progs, X, y, steps=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ag.tune_constants(progs, X, y, steps=20, lr=0.05)
    torch.cuda.synchronize()
    adam_s = time.perf_counter() - t0
    ok = torch.isfinite(res.fitness_before) & torch.isfinite(res.fitness_after)
    improved = float((res.fitness_after[ok] < res.fitness_before[ok]).double().mean().item())
    return {"workload": "adjoint: N=4096, L~U{8..64}, 1..8 constants, D=5, M=100000, MSE (and 1 - r^2)",
            "fwd_gpops": round(fwd, 2), "fwd_adjoint_gpops": round(both, 2),
            "adjoint_cost_vs_fwd": round(fwd / both, 3),
            "corr_fwd_gpops": round(fwd_c, 2), "corr_fwd_adjoint_gpops": round(both_c, 2),
            "adam_20_steps_ms": round(adam_s * 1e3, 2),
            "adam_gpops": round(nc * 21 / adam_s / 1e9, 2),
            "adam_programs_improved": round(improved, 3)}


def scores_bench(steps: int, warmup: int):
    """The paper's scores (Eq. 3 summed over cases, Eq. 2) on the plain-mid
    population with targets undefined on a quarter of the domain (same
    shape: D=5, M=100000); GPop/s as for the main metric."""
    import torch
    from paper_2603_12292_amd import api
    from paper_2603_12292_amd import workloads as wl
    w = wl.config_mid()
    data = wl.invalid_target_dataset(2609, 100_000, 5)
    progs = api.DevicePrograms.from_programset(w.programs, "cuda:0")
    X = torch.from_numpy(data.X).cuda()
    y = torch.from_numpy(data.y).cuda()
    nc = w.programs.node_count() * data.M

    def rate(kind):
        for _ in range(warmup):
            api.evaluate_score(progs, X, y, kind, 1000.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            api.evaluate_score(progs, X, y, kind, 1000.0)
        torch.cuda.synchronize()
        return nc * steps / (time.perf_counter() - t0) / 1e9

    return {"workload": "scores: plain-mid programs, y = log(x0 - 2)(1 + x1/4) (NaN on x0 < 2), M=100000, S=1000",
            "point_gpops": round(rate("point"), 2), "r4_gpops": round(rate("r4"), 2)}


def paper_shape_bench(steps: int, warmup: int):
    """The paper's regime: 2^20 programs (plain-mid x256, L~U{5..64}) on
    512 cases, per whole-population evaluation (decode, staging,
    interpreter, reductions) for the MSE, 1 - r^2 and the paper's two
    scores; GPop/s as for the main metric."""
    import torch
    from paper_2603_12292_amd import api
    from paper_2603_12292_amd import workloads as wl
    w = wl.config_paper_shape()
    progs = api.DevicePrograms.from_programset(w.programs, "cuda:0")
    X = torch.from_numpy(w.data.X).cuda()
    y = torch.from_numpy(w.data.y).cuda()
    nc = w.programs.node_count() * w.data.M
    out = {"workload": w.name}
    for kind in ("mse", "corr", "point", "r4"):
        def call():
            if kind in ("mse", "corr"):
                api.evaluate(progs, X, y, kind)
            else:
                api.evaluate_score(progs, X, y, kind, 1000.0)
        for _ in range(max(1, warmup)):
            call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = max(1, steps // 2)
        for _ in range(n):
            call()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n
        out[f"{kind}_ms"] = round(dt * 1e3, 3)
        out[f"{kind}_gpops"] = round(nc / dt / 1e9, 2)
    return out


# The paper's population schedule under correlation fitness (its parameter
# table): 5M individuals before generation 5, 3M before 10, 1M before 15,
# 500k before 20, 250k from then on.
PAPER_CORR_SCHEDULE = ((5, 5_000_000), (10, 3_000_000), (15, 1_000_000), (20, 500_000), (None, 250_000))


def paper_pop_size(g: int) -> int:
    for end, n in PAPER_CORR_SCHEDULE:
        if end is None or g < end:
            return n
    raise AssertionError


def paper_loop_bench(generations: int, op_set: int = 0):
    """The paper's evolutionary loop at its own sizes: ramped half-and-half
    initial population (depths 2..5, max length 64) over the 9 base
    operators (op_set 0) or the paper's 16 (op_set 1), correlation fitness
    (1 - r^2) on 512 cases (D = 5), microcosm selection (sample 100, keep
    0.5) and mutation-only variation, the population following the paper's
    correlation schedule; everything on the GPU, one stream.  Reports the
    time per generation (evaluation, selection + variation) at each
    population size."""
    import torch
    from paper_2603_12292_amd import api
    from paper_2603_12292_amd import workloads as wl
    data = wl.config_paper_shape().data
    X = torch.from_numpy(data.X).cuda()
    y = torch.from_numpy(data.y).cuda()
    params = api.GenParams(tournament=1, p_crossover=0.0, p_mutation=1.0, max_len=64, max_consts=8,
                           init_depth_min=2, init_depth_max=5, op_set=op_set)
    D, seed = data.D, 2612
    ctx = api.context(0)
    init = api.init_population(paper_pop_size(0), D, params, seed, ctx=ctx)

    def run(ev, lens):
        pop = init
        for g in range(generations):
            e0, e1, e2 = ev[g]
            e0.record()
            fit = api.evaluate(pop.programs(), X, y, "corr", ctx=ctx)
            e1.record()
            lens.append(pop.len.to(torch.int64).sum())
            pop = api.generation_microcosm(pop.programs(), fit, params, D, seed, g + 1, paper_pop_size(g + 1),
                                           sample=100, keep=0.5, ctx=ctx)
            e2.record()

    # an untimed pass of the whole schedule first: evaluator tuning, the
    # workspace and torch's allocator cache reach their final sizes (the
    # timed pass repeats it bit for bit: same seed, same initial population)
    mk = lambda: [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(generations)]
    run(mk(), [])
    torch.cuda.synchronize()
    ev = mk()
    lens = []
    t0 = time.perf_counter()
    run(ev, lens)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tokens = [int(t) for t in torch.stack(lens).cpu()]
    phases = {}
    for g in range(generations):
        n = paper_pop_size(g)
        e0, e1, e2 = ev[g]
        ph = phases.setdefault(n, {"generations": 0, "eval_ms": 0.0, "select_vary_ms": 0.0, "node_cases": 0})
        ph["generations"] += 1
        ph["eval_ms"] += e0.elapsed_time(e1)
        ph["select_vary_ms"] += e1.elapsed_time(e2)
        ph["node_cases"] += tokens[g] * data.M
    rows = []
    for n, ph in phases.items():
        k = ph["generations"]
        rows.append({"population": n, "generations": k, "eval_ms": round(ph["eval_ms"] / k, 3),
                     "select_vary_ms": round(ph["select_vary_ms"] / k, 3),
                     "generation_ms": round((ph["eval_ms"] + ph["select_vary_ms"]) / k, 3),
                     "eval_gpops": round(ph["node_cases"] / (ph["eval_ms"] / 1e3) / 1e9, 2)})
    ops = "the paper's 16 operators" if op_set == 1 else "the 9 base operators"
    return {"workload": f"paper loop: correlation fitness, M={data.M}, D={D}, ramped half-and-half depths 2..5 "
                        f"(max length 64), {ops}, microcosm selection (sample 100, keep 0.5), mutation only, "
                        f"population 5M/3M/1M/500k/250k at generations 0/5/10/15/20",
            "generations": generations, "wall_s": round(wall, 3), "phases": rows,
            "mean_len_first": round(tokens[0] / paper_pop_size(0), 2),
            "mean_len_last": round(tokens[-1] / paper_pop_size(generations - 1), 2)}


def ragged_bench(steps: int, warmup: int):
    """The 64-problem ragged workload (1024 programs each, L~U{5..96},
    D~U{1..9}, M=round(10^U(3,6)), MSE): one batched call (a replayed HIP
    graph over all problems) against 64 separate beagle_eval calls, both on
    torch's current stream, inputs resident."""
    import torch
    from paper_2603_12292_amd import api
    from paper_2603_12292_amd import workloads as wl
    ws = wl.ragged_problems()
    dev = [(api.DevicePrograms.from_programset(w.programs, "cuda:0"), torch.from_numpy(w.data.X).cuda(),
            torch.from_numpy(w.data.y).cuda()) for w in ws]
    out = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p, _, _ in dev]
    nc = sum(w.programs.node_count() * w.data.M for w in ws)
    ctx = api.context(0)

    def batched():
        api.evaluate_batched(dev, "mse", out=out, ctx=ctx)

    def sequential():
        for p, X, y in dev:
            api.evaluate(p, X, y, "mse", ctx=ctx)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    tb = timed(batched)
    ts = timed(sequential)
    return {"workload": "ragged: 64 problems x 1024 programs, L~U{5..96}, D~U{1..9}, M=round(10^U(3,6)), MSE",
            "node_cases": nc, "batched_ms": round(tb * 1e3, 3), "sequential_ms": round(ts * 1e3, 3),
            "batched_gpops": round(nc / tb / 1e9, 2), "sequential_gpops": round(nc / ts / 1e9, 2),
            "batched_speedup": round(ts / tb, 3)}


def generation_bench(generations: int):
    """The generation loop: ramped half-and-half N=16384 (depths 2..6, max
    length 128), D=9, M=10^6, MSE; per generation one evaluation and one
    selection + variation step (tournament 4, crossover 0.9, mutation 0.1),
    everything on the GPU.  GPop/s counts the evaluations' node-cases."""
    import torch
    from paper_2603_12292_amd import api
    from paper_2603_12292_amd import workloads as wl
    data = wl.generation_dataset()
    X = torch.from_numpy(data.X).cuda()
    y = torch.from_numpy(data.y).cuda()
    params = api.GenParams()
    N, D, seed = 16384, data.D, 2606
    ctx = api.context(0)
    pop = api.init_population(N, D, params, seed, ctx=ctx)
    spare = api.Slots.empty(N, params.max_len, params.max_consts, "cuda")
    api.evaluate(pop.programs(), X, y, "mse", ctx=ctx)  # tunes the bucket of generation 0
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(generations + 1)]
    lens = []
    t0 = time.perf_counter()
    for g in range(generations + 1):
        e0, e1, e2 = ev[g]
        e0.record()
        fit = api.evaluate(pop.programs(), X, y, "mse", ctx=ctx)
        e1.record()
        lens.append(pop.len.to(torch.int64).sum())
        if g < generations:
            api.generation(pop.programs(), fit, params, D, seed, g + 1, out=spare, ctx=ctx)
            pop, spare = spare, pop
        e2.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = [a.elapsed_time(b) for a, b, _ in ev]
    gen_ms = [b.elapsed_time(c) for _, b, c in ev[:-1]]
    tokens = [int(t) for t in torch.stack(lens).cpu()]
    nc = sum(tokens) * data.M
    return {"workload": f"generation loop: N={N}, ramped half-and-half depths 2..6, max length 128, D={D}, "
                        f"M={data.M}, MSE, tournament 4, crossover 0.9, mutation 0.1",
            "evaluations": generations + 1, "wall_s": round(wall, 3),
            "eval_ms_mean": round(float(np.mean(ev_ms)), 3), "generation_step_ms_mean": round(float(np.mean(gen_ms)), 4),
            "eval_gpops": round(nc / (sum(ev_ms) / 1e3) / 1e9, 2), "loop_gpops": round(nc / wall / 1e9, 2),
            "mean_len_first": round(tokens[0] / N, 2), "mean_len_last": round(tokens[-1] / N, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-programs", type=int, default=4096)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--no-scores", action="store_true", help="skip the paper's Eq. 2 / Eq. 3 score rates")
    ap.add_argument("--no-paper-shape", action="store_true", help="skip the 2^20-program x 512-case rates")
    ap.add_argument("--generations", type=int, default=50, help="generation-loop length (0 = skip)")
    ap.add_argument("--paper-loop", type=int, default=25,
                    help="generations of the paper's own loop at its population schedule (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (one process, one device)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_12292_amd import api
    from paper_2603_12292_amd import workloads as wl

    w = wl.config_mid()
    ps = w.programs
    # the CPU oracle first: its worker processes are forked before this
    # process starts the GPU runtime (forking after that is not safe)
    cpu = cpu_baseline(w, 1, args.cpu_programs) if not args.no_cpu_baseline else None
    dev = torch.device("cuda:0")
    progs = api.DevicePrograms.from_programset(ps, dev)
    X = torch.from_numpy(w.data.X).to(dev)
    y = torch.from_numpy(w.data.y).to(dev)
    ctx = api.context(0)
    nodes = ps.node_count()
    M = w.data.M

    for _ in range(args.warmup):
        api.evaluate(progs, X, y, "corr", ctx=ctx)
    torch.cuda.synchronize()
    ctx.enable_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fit = api.evaluate(progs, X, y, "corr", ctx=ctx)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_n = ctx.kernel_time()
    ctx.enable_timing(False)
    dt = t1 - t0
    gpops = nodes * M * args.steps / dt / 1e9
    assert np.isfinite(fit.cpu().numpy()).sum() > 0

    width = ctx.tile_width("corr", w.data.D, M, int(ps.tokens.size), ps.n)
    kernel = f"k_eval_class<1, 0, {0 if width == 8 else 1}>"
    k_avg_s = k_ms / 1e3 / max(k_n, 1)
    fn = function_nodes(ps)
    alg_ops = fn * M                       # one fp32 op per operator application
    achieved = alg_ops / k_avg_s
    counters = committed_counters(kernel)
    traffic = counters.get("hbm_bytes_per_launch")
    out = {
        "metric": "GPop/s (program-node x fitness-case evals/s), fwd and fwd+adjoint, 1 MI355X",
        "value": round(gpops, 2),
        "unit": "GPop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (binary64 sums)",
        "data": "synthetic",
        "config": {"workload": "plain-mid: N=4096 programs, L~U{5..64}, D=5, M=100000, X~U(1,10), "
                               "20-token target, correlation fitness 1-r^2",
                   "programs": ps.n, "fitness_cases": M, "nodes": nodes, "kind": "corr"},
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 4), "peak": round(PEAK_LANE_OPS / 1e12, 2),
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_LANE_OPS, 4),
                     "traffic": traffic,
                     "kernel": f"{kernel}: correlation fitness, register need <= 4, {width} cases per lane",
                     "kernel_ms": round(k_avg_s * 1e3, 4), "alg_ops_per_launch": alg_ops,
                     "kernel_gpops": round(nodes * M / k_avg_s / 1e9, 2),
                     "valu_issue_frac": (round(counters["valu_issue_frac"], 4)
                                         if "valu_issue_frac" in counters else None)},
    }
    if not args.no_adjoint:
        out["adjoint"] = adjoint_bench(args.steps, args.warmup)
    if not args.no_scores:
        out["scores"] = scores_bench(args.steps, args.warmup)
    if not args.no_paper_shape:
        out["paper_shape"] = paper_shape_bench(args.steps, args.warmup)
    if not args.no_ragged:
        out["ragged"] = ragged_bench(max(1, args.steps // 4), max(1, args.warmup))
    if args.generations > 0:
        out["generation_loop"] = generation_bench(args.generations)
    if args.paper_loop > 0:
        out["paper_loop"] = paper_loop_bench(args.paper_loop)
        out["paper_loop_16_ops"] = paper_loop_bench(args.paper_loop, op_set=1)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
