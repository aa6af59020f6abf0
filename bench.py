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

# MI355X's published fp32 vector peak (256 CUs x 256 flop/clock x 2.4 GHz;
# it counts a packed two-wide FMA as four flops): the roofline denominator.
PEAK_FP32 = 157.3e12
# its non-packed fp32 lane-operation issue rate, 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz: the denominator of the issue fraction measured by counters
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
HBM_PEAK = 8.0e12
# binary64 operations of the fitness epilogue per program and case
# (MSE: difference, square-add, mask; 1 - r^2: u, w, three sums)
EPILOGUE_OPS = {"mse": 3, "corr": 5}


def function_nodes(ps) -> int:
    ops = ps.tokens & 0xFF
    return int(np.count_nonzero((ops < 9) | (ops > 10)))


def committed_counters(kernel: str) -> dict:
    """Counter figures of the interpreter kernel from the committed profile
    summary (HBM bytes per launch, VALU and SALU instructions), or {} when
    the kernel source changed since they were taken or they are of another
    tile-width variant."""
    from paper_2603_12292_amd.profiling import source_hash
    path = os.path.join(ROOT, "profiles", "k_eval_class_corr_plain_mid_traffic.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash() or rec.get("kernel") != kernel:
        return {}
    return rec


def job_cores() -> int:
    """Host cores this job may use: its affinity mask, limited by the thread
    allotment it runs under (OMP_NUM_THREADS, which a shared GPU machine sets to
    the job's CPU share)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return n


def _pool_map(fn, items, cores):
    """fn over items in a process pool (fork: called before this process
    starts the GPU runtime), results in order."""
    if cores <= 1:
        return [fn(x) for x in items]
    import multiprocessing as mp
    before = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        with mp.get_context("fork").Pool(cores) as pool:
            return pool.map(fn, items, chunksize=1)
    finally:
        if before is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = before


def _oracle_eval(ps, data, kind_id, cores, subset=None):
    """(seconds, fitness[...], node-cases) of the binary64 oracle."""
    from oracle import population as opop
    idx = list(range(ps.n)) if subset is None else list(subset)
    nodes = int(ps.tok_len[idx].astype(np.int64).sum())
    t0 = time.perf_counter()
    f, _ = opop.evaluate_population(ps.tokens, ps.tok_offset, ps.tok_len, ps.consts, ps.const_offset,
                                    ps.const_count, data.X, data.y, kind_id, "o64", subset=idx, processes=cores)
    return time.perf_counter() - t0, f, nodes * data.M


def _grad_one(args):
    from oracle import grad as og
    toks, consts, X, y = args
    return og.mse_and_grad(toks, consts, X, y)


def cpu_baselines(w, cores, ragged):
    """The binary64 CPU oracle, timed on this host before the GPU runtime
    starts: the benchmark workload in full (the contract's cpu_baseline,
    also kept for the parity statistics), and the other workloads on the
    bounded samples stated in each entry."""
    from paper_2603_12292_amd import workloads as wl
    dt, f64, nc = _oracle_eval(w.programs, w.data, 1, cores)
    main = {"value": nc / dt / 1e9, "unit": "GPop/s", "cores": cores, "kind": "oracle",
            "sample": f"{w.programs.n} of {w.programs.n} programs, all {w.data.M} cases, correlation fitness, "
                      f"float64 oracle, {dt:.1f} s wall"}
    other = {}
    tiny = wl.config_tiny()
    for kid, name in ((0, "mse"), (1, "corr")):
        d, _, n = _oracle_eval(tiny.programs, tiny.data, kid, cores)
        other[f"plain_tiny_{name}"] = {"value": round(n / d / 1e9, 4), "unit": "GPop/s", "cores": cores,
                                       "sample": f"all 256 programs x 1000 cases, {d:.2f} s"}
    d, _, n = _oracle_eval(w.programs, w.data, 0, cores, subset=range(0, w.programs.n, 8))
    other["plain_mid_mse"] = {"value": round(n / d / 1e9, 4), "unit": "GPop/s", "cores": cores,
                              "sample": f"SUBSET: 512 of 4096 programs (every 8th), all 100000 cases, {d:.2f} s"}
    # generation loop: one generation's evaluation on a program sample,
    # scaled to the population, plus the oracle's whole variation step
    from oracle import gp
    gd = wl.generation_dataset()
    params = gp.GenParams()
    pop = gp.init_population(16384, gd.D, params, 2606)
    ps0 = wl.pack_programs(pop)
    sub = list(range(0, 16384, 256))
    d_e, f_e, n_e = _oracle_eval(ps0, gd, 0, cores, subset=sub)
    fit = np.arange(16384, dtype=np.float64) * 1e-3   # any ordering: the step's cost
    fit[sub] = f_e
    t0 = time.perf_counter()
    gp.generation([t for t, _ in pop], [c for _, c in pop], fit, gd.D, params, 2606, 1)
    d_v = time.perf_counter() - t0
    eval_s = d_e * 16384 / len(sub)
    other["generation_loop"] = {
        "eval_gpops": round(n_e / d_e / 1e9, 4), "unit": "GPop/s", "cores": cores,
        "s_per_generation": round(eval_s + d_v, 2), "s_51_evaluations_50_steps": round(51 * eval_s + 50 * d_v, 1),
        "sample": f"EXTRAPOLATED: generation 0 evaluated on 64 of 16384 programs (every 256th) x 10^6 cases "
                  f"({d_e:.2f} s) scaled to the population, one whole variation step (16384 children, one core, "
                  f"{d_v:.2f} s); the loop's 51 evaluations and 50 steps scaled from these"}
    # ragged batching: every 8th problem, every 32nd program of it
    nc_all = sum(q.programs.node_count() * q.data.M for q in ragged)
    tot_s = tot_n = 0
    for q in ragged[::8]:
        d, _, n = _oracle_eval(q.programs, q.data, 0, cores, subset=range(0, q.programs.n, 32))
        tot_s += d
        tot_n += n
    other["ragged"] = {"value": round(tot_n / tot_s / 1e9, 4), "unit": "GPop/s", "cores": cores,
                       "s_whole_workload": round(tot_s * nc_all / tot_n, 1),
                       "sample": f"SUBSET: 8 of 64 problems (every 8th) x 32 of 1024 programs (every 32nd), "
                                 f"{tot_n:.3g} of {nc_all:.3g} node-cases ({tot_s:.1f} s); the whole-workload "
                                 f"time scaled by node-cases"}
    # differentiation: forward and forward + gradient on 64 programs
    dw = wl.config_differentiation()
    sub = list(range(0, dw.programs.n, 64))
    d_f, _, n_f = _oracle_eval(dw.programs, dw.data, 0, cores, subset=sub)
    args = []
    for p in sub:
        t, c = dw.programs.program(p)
        args.append((t, c, dw.data.X, dw.data.y))
    t0 = time.perf_counter()
    _pool_map(_grad_one, args, cores)
    d_g = time.perf_counter() - t0
    other["differentiation"] = {"fwd_gpops": round(n_f / d_f / 1e9, 4),
                                "fwd_adjoint_gpops": round(n_f / d_g / 1e9, 4), "unit": "GPop/s", "cores": cores,
                                "sample": f"SUBSET: 64 of 4096 programs (every 64th) x 100000 cases, MSE: forward "
                                          f"{d_f:.2f} s, fitness and constant gradients {d_g:.2f} s"}
    return main, other, f64


def parity_stats(gpu, f64_fresh, w, kind_id):
    """Gate statistics of the GPU fitness of every program of the benchmark
    workload against the oracle's stored values (tests/golden), after
    checking that the oracle run above reproduces the stored binary64 ones."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import gates
    import golden_mid
    refs = golden_mid.load(w)[kind_id]
    same = None if f64_fresh is None else bool(np.array_equal(f64_fresh, refs.f64, equal_nan=True))
    s = gates.check(gpu, refs, kind_id, w.data.y, max_ill_frac=1.0, max_unchecked_frac=1.0, min_value=0)
    return {"programs": int(len(gpu)), "finite": s.n_finite, "value_gate_1e-5": s.n_value,
            "ill_conditioned": s.n_ill, "envelope_gate": s.n_env, "bound_vacuous": s.n_vacuous,
            "unchecked": s.n_unchecked, "max_err_over_gate": round(float(s.max_gate), 4),
            "all_gates_pass": True, "oracle_rerun_matches_stored": same}


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


def selection_bench(populations=(1_000_000, 5_000_000), reps: int = 20):
    """The context of the paper's section 2.1.6 (microcosm selection against
    a full ranking): per population size, the microcosm selection pass
    (threshold from a 100-draw sample, survivor list; beagle_generation_
    microcosm without children) against a full ranking of the same float64
    fitness on the GPU (torch.sort, a device radix sort, then the better
    half's indices as the survivor list), both timed with events, fitness
    resident (uniform values with 1 % NaN)."""
    import torch
    from paper_2603_12292_amd import api
    ctx = api.context(0)
    params = api.GenParams(tournament=1, p_crossover=0.0, p_mutation=1.0, max_len=64, max_consts=8,
                           init_depth_min=2, init_depth_max=5)
    rows = []
    for n in populations:
        g = torch.Generator(device="cuda").manual_seed(7)
        fit = torch.rand(n, dtype=torch.float64, device="cuda", generator=g)
        fit[torch.rand(n, device="cuda", generator=g) < 0.01] = float("nan")
        # parents are not read without children: a one-token program per slot
        toks = torch.full((n,), 9, dtype=torch.int16, device="cuda")
        progs = api.DevicePrograms(toks, torch.arange(n, dtype=torch.int64, device="cuda"),
                                   torch.ones(n, dtype=torch.int32, device="cuda"),
                                   torch.zeros(1, dtype=torch.float32, device="cuda"),
                                   torch.zeros(n, dtype=torch.int64, device="cuda"),
                                   torch.zeros(n, dtype=torch.int32, device="cuda"))

        def micro(i):
            return api.generation_microcosm(progs, fit, params, 1, 11, i, 0, sample=100, keep=0.5,
                                            with_selection=True, ctx=ctx)

        def ranking(i):
            order = torch.sort(fit).indices   # ascending, NaN last
            return order[: n // 2]

        out = {}
        for name, fn in (("microcosm_select_ms", micro), ("full_ranking_ms", ranking)):
            for i in range(3):
                fn(i)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(reps):
                fn(i)
            e1.record()
            torch.cuda.synchronize()
            out[name] = round(e0.elapsed_time(e1) / reps, 4)
        _, _, ns = micro(0)
        out.update({"population": n, "microcosm_survivors": int(ns.item()),
                    "ranking_over_microcosm": round(out["full_ranking_ms"] / out["microcosm_select_ms"], 1)})
        rows.append(out)
    return {"workload": "selection on float64 fitness (uniform, 1 % NaN): microcosm (sample 100, keep 0.5) "
                        "against a full device sort keeping the better half", "rows": rows}


def ragged_bench(ws, steps: int, warmup: int):
    """The 64-problem ragged workload (1024 programs each, L~U{5..96},
    D~U{1..9}, M=round(10^U(3,6)), MSE): one batched call (a replayed HIP
    graph over all problems) against 64 separate beagle_eval calls, both on
    torch's current stream, inputs resident."""
    import torch
    from paper_2603_12292_amd import api
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


def plain_rate(w, kind, steps, warmup, ctx):
    """GPop/s of whole beagle_eval calls on one workload (inputs resident)."""
    import torch
    from paper_2603_12292_amd import api
    progs = api.DevicePrograms.from_programset(w.programs, "cuda:0")
    X = torch.from_numpy(w.data.X).cuda()
    y = torch.from_numpy(w.data.y).cuda()
    for _ in range(max(1, warmup)):
        api.evaluate(progs, X, y, kind, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fit = api.evaluate(progs, X, y, kind, ctx=ctx)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return w.programs.node_count() * w.data.M / dt / 1e9, dt, fit.cpu().numpy()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--main-only", action="store_true",
                    help="only the main line (every other line and the CPU baseline skipped): the run whose "
                         "kernel trace gives the interpreter's average launch duration")
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

    from paper_2603_12292_amd import workloads as wl

    w = wl.config_mid()
    ps = w.programs
    if args.main_only:
        args.no_cpu_baseline = True
    ragged = wl.ragged_problems() if not (args.no_ragged and args.no_cpu_baseline) else None
    # the CPU oracle first: its worker processes are forked before this
    # process starts the GPU runtime (forking after that is not safe)
    cpu = cpu_baselines(w, job_cores(), ragged) if not args.no_cpu_baseline else None

    import torch
    from paper_2603_12292_amd import api
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
    fit = fit.cpu().numpy()
    assert np.isfinite(fit).sum() > 0

    width = ctx.tile_width("corr", w.data.D, M, int(ps.tokens.size), ps.n)
    kernel = f"k_eval_class<1, 0, {0 if width == 8 else 1}>"
    k_avg_s = k_ms / 1e3 / max(k_n, 1)
    fn = function_nodes(ps)
    # algorithmic work of one launch: one operation per operator application
    # (binary or unary; terminals move data) plus the binary64 epilogue per
    # program and case
    alg_ops = fn * M + EPILOGUE_OPS["corr"] * ps.n * M
    achieved = alg_ops / k_avg_s
    counters = committed_counters(kernel)
    traffic = counters.get("hbm_bytes_per_launch")
    node_cases = nodes * M
    valu = counters.get("valu_insts_per_launch")
    salu = counters.get("salu_insts_per_launch")
    wave_tiles = -(-M // (64 * width))           # passes of one wave over the cases of a program
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
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 4), "peak": round(PEAK_FP32 / 1e12, 1),
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32, 4),
                     "traffic": traffic,
                     "kernel": f"{kernel}: correlation fitness, register need <= 4, {width} cases per lane",
                     "kernel_ms": round(k_avg_s * 1e3, 4), "alg_ops_per_launch": alg_ops,
                     "kernel_gpops": round(node_cases / k_avg_s / 1e9, 2),
                     "valu_issue_frac": (round(counters["valu_issue_frac"], 4)
                                         if "valu_issue_frac" in counters else None),
                     "valu_issue_peak_lane_ops": round(PEAK_LANE_OPS / 1e12, 2),
                     "valu_lane_ops_per_node_case": round(valu * 64 / node_cases, 3) if valu else None,
                     "salu_insts_per_node_per_wave": (round(salu / (nodes * wave_tiles), 2) if salu else None)},
    }
    if cpu is not None:
        main_cpu, other_cpu, f64 = cpu
        out["parity"] = parity_stats(fit, f64, w, 1)
    if args.main_only:
        print(json.dumps(out), flush=True)
        return
    mid_mse, _, fit_mse = plain_rate(w, "mse", args.steps, args.warmup, ctx)
    out["plain_mid_mse"] = {"workload": "plain-mid, MSE", "gpops": round(mid_mse, 2)}
    if cpu is not None:
        out["plain_mid_mse"]["parity"] = parity_stats(fit_mse, None, w, 0)
    tiny = wl.config_tiny()
    out["plain_tiny"] = {"workload": tiny.name}
    for kind in ("mse", "corr"):
        g, d, _ = plain_rate(tiny, kind, args.steps, args.warmup, ctx)
        out["plain_tiny"][f"{kind}_gpops"] = round(g, 3)
        out["plain_tiny"][f"{kind}_us"] = round(d * 1e6, 1)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_bench(args.steps, args.warmup)
    if not args.no_scores:
        out["scores"] = scores_bench(args.steps, args.warmup)
    if not args.no_paper_shape:
        out["paper_shape"] = paper_shape_bench(args.steps, args.warmup)
    if not args.no_ragged:
        out["ragged"] = ragged_bench(ragged, max(1, args.steps // 4), max(1, args.warmup))
    if args.generations > 0:
        out["generation_loop"] = generation_bench(args.generations)
    if args.paper_loop > 0:
        out["paper_loop"] = paper_loop_bench(args.paper_loop)
        out["paper_loop_16_ops"] = paper_loop_bench(args.paper_loop, op_set=1)
        out["selection"] = selection_bench()
    if cpu is not None:
        out["cpu_baseline"] = main_cpu
        out["cpu_baselines_other"] = other_cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
