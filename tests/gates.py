"""Parity gates between GPU fitness and the CPU oracle.

Three gates, applied to every program of a comparison:

Classification gate: the GPU fitness class (finite / +inf / nan) equals the
class the fp32-emulating oracle (O32e) gives; an fp32 evaluation can
overflow where binary64 does not, so the classes come from O32e, not from
the binary64 oracle.

Envelope gate (every program finite on both sides): |F_gpu - F_O32e| <=
B (1 + 1e-6) + 1e-8 |F_O32e| + atol, with B the bound of oracle.bound: how
far the fitness can move when every approximate operator's result carries
its stated error (sin, cos, exp, log within 2 ulp, sqrt faithful, the
library's tan, asin, acos, atan, tanh within 4 ulp) and every correctly
rounded operator with an inexact operand re-rounds (a running error bound
per case, combined exactly through the MSE and through r of Eq. 1);
1e-8 |F| covers the binary64 summation order.  Programs whose bound is
infinite (on some case a value may reach a pole or a branch point of an
operator within its error, or F is the convention for a constant output)
are counted as "vacuous"; those among them that the value gate does not
cover either are counted as unchecked and bounded in number.

Output gate (the programs neither gate below or above covers: ill
conditioned with a vacuous bound): the GPU's own per-case outputs (from
beagle_predict, the same interpreter code) on every case whose per-case
bound is finite lie within it of O32e's, and the GPU fitness equals the
oracle's fitness of those outputs (binary64 summation order aside) -- the
reduction checked exactly, the interpreter everywhere a bound exists.

Value gate (the claim: within 1e-5 of the binary64 oracle):
|F_gpu - F_O64| <= 1e-5 |F_O64| + atol for every program that is finite in
both and well conditioned: its fitness moves by at most 1e-6 |F_O64| + atol
(a tenth of the gate) when every token is rounded to fp32 (O32e) and in two
runs where every approximate operator's result is also perturbed by a few
ulps (O32p, two seeds).  Finite programs outside that set ("ill
conditioned", e.g. exp of a large argument under MSE) are still held to the
envelope gate; their number is bounded per workload.

atol = 1e-10 * mean(y^2) for MSE, 1e-9 for correlation fitness.
"""
import math
from typing import List, NamedTuple

import numpy as np

from oracle import bound as obound
from oracle import fitness as ofit
from oracle import population as opop

RTOL = 1e-5
RTOL_COND = 1e-6
ENV_RTOL = 1e-8
# relative error bound of the library's division against the correctly
# rounded quotient of o32e: faithful (within 1 ulp of the exact quotient),
# o32e within 1/2: 1.5 ulp < 2^-22
DIV_EPS = 2.0 ** -22


def atol(kind, y):
    y64 = np.asarray(y, dtype=np.float64)
    return 1e-10 * float(np.mean(y64 * y64)) if kind == ofit.MSE else 1e-9


def oracle(ps, X, y, kind, mode, subset=None, processes=None, seed=0):
    return opop.evaluate_population(ps.tokens, ps.tok_offset, ps.tok_len, ps.consts, ps.const_offset,
                                    ps.const_count, X, y, kind, mode, subset=subset, processes=processes,
                                    seed=seed, div_eps=DIV_EPS)


class Refs(NamedTuple):
    """The oracle's values for a list of programs: binary64 fitness, status,
    fp32-emulated fitness, perturbed fp32 fitness (two seeds), first-order
    bound of the fp32 evaluation."""
    f64: np.ndarray
    status: np.ndarray
    f32: np.ndarray
    pert: List[np.ndarray]
    bound: np.ndarray

    def take(self, idx):
        idx = np.asarray(idx)
        return Refs(self.f64[idx], self.status[idx], self.f32[idx], [p[idx] for p in self.pert], self.bound[idx])


def references(ps, X, y, kind, subset=None, processes=None) -> Refs:
    f64, s64 = oracle(ps, X, y, kind, "o64", subset, processes)
    f32, _ = oracle(ps, X, y, kind, "o32e", subset, processes)
    pert = [oracle(ps, X, y, kind, "o32p", subset, processes, seed=s)[0] for s in (1, 2)]
    b, _ = oracle(ps, X, y, kind, "bound", subset, processes)
    return Refs(f64, s64, f32, pert, b)


class Stats(NamedTuple):
    n_value: int     # programs held to the 1e-5 value gate against O64
    n_ill: int       # finite programs outside it (ill conditioned)
    n_env: int       # finite programs held to the envelope gate (finite bound)
    n_vacuous: int   # finite programs whose bound is infinite
    n_finite: int    # programs finite in the fp32-emulating oracle
    n_unchecked: int  # finite programs under neither value gate (ill conditioned and vacuous)
    max_gate: float  # largest |F_gpu - F_O64| / (1e-5 |F_O64| + atol) over the value-gated programs
    unchecked: tuple = ()  # indices of the unchecked programs (for the output gate)

    @property
    def n_checked(self) -> int:
        """finite programs under at least one value gate"""
        return self.n_finite - self.n_unchecked


def check(gpu, refs: Refs, kind, y, max_ill_frac=0.05, label="", max_unchecked_frac=0.05, min_value=1) -> Stats:
    """Apply the three gates to every program; returns the counts."""
    gpu = np.asarray(gpu, dtype=np.float64)
    f64, f32e, pert, bound = refs.f64, refs.f32, refs.pert, refs.bound
    at = atol(kind, y)
    cls_gpu = [ofit.classify(v) for v in gpu]
    cls_32 = [ofit.classify(v) for v in f32e]
    bad_cls = [i for i in range(len(gpu)) if cls_gpu[i] != cls_32[i]]
    assert not bad_cls, (label, "classification", [(i, gpu[i], f32e[i], f64[i]) for i in bad_cls[:10]])
    n_val = n_ill = n_env = n_vac = n_unc = 0
    unc = []
    max_gate = 0.0
    bad_val, bad_env = [], []
    for i in range(len(gpu)):
        if not (math.isfinite(gpu[i]) and math.isfinite(f32e[i])):
            continue
        vacuous = math.isinf(bound[i])
        if vacuous:
            n_vac += 1
        else:
            n_env += 1
            lim = bound[i] * (1.0 + 1e-6) + ENV_RTOL * abs(f32e[i]) + at
            if not abs(gpu[i] - f32e[i]) <= lim:
                bad_env.append((i, gpu[i], f32e[i], bound[i]))
        if not math.isfinite(f64[i]) or not all(math.isfinite(p[i]) for p in pert) or \
                max([abs(f32e[i] - f64[i])] + [abs(p[i] - f64[i]) for p in pert]) > RTOL_COND * abs(f64[i]) + at:
            n_ill += 1
            if vacuous:
                n_unc += 1
                unc.append(i)
            continue
        n_val += 1
        err = abs(gpu[i] - f64[i])
        max_gate = max(max_gate, err / (RTOL * abs(f64[i]) + at))
        if err > RTOL * abs(f64[i]) + at:
            bad_val.append((i, gpu[i], f64[i], f32e[i]))
    assert not bad_env, (label, "envelope", bad_env[:10])
    assert not bad_val, (label, "value", bad_val[:10])
    finite = sum(1 for c in cls_32 if c == "finite")
    assert n_ill <= max_ill_frac * max(finite, 1) + 2, (label, "too many ill-conditioned", n_ill, finite)
    assert n_unc <= max_unchecked_frac * max(finite, 1) + 2, (label, "too many programs unchecked", n_unc, finite)
    assert n_val >= min_value, (label, "no program value-checked", n_val, finite)
    return Stats(n_val, n_ill, n_env, n_vac, finite, n_unc, max_gate, tuple(unc))


def check_outputs(programs, X, y, kind, outs, fitness, label=""):
    """The output gate for a list of (tokens, consts) programs with the GPU's
    per-case outputs outs[k] (binary32) and fitness[k]; returns (cases
    checked, cases without a bound)."""
    at = atol(kind, y)
    n_ok = n_free = 0
    for k, (toks, consts) in enumerate(programs):
        values, _, d, _ = obound.case_bounds(toks, consts, X, div_eps=DIV_EPS)
        y32, b = values[-1], d[-1]
        out = np.asarray(outs[k], dtype=np.float64)
        fin = np.isfinite(b)
        bad = np.flatnonzero(fin & ~(np.abs(out - y32) <= b * (1.0 + 1e-6)))
        assert bad.size == 0, (label, "output", k, [(int(i), out[i], y32[i], b[i]) for i in bad[:5]])
        n_ok += int(fin.sum())
        n_free += int((~fin).sum())
        f_own = ofit.fitness(kind, out, y)
        assert ofit.classify(f_own) == ofit.classify(fitness[k]), (label, "output fitness class", k)
        if math.isfinite(f_own):
            assert abs(fitness[k] - f_own) <= ENV_RTOL * abs(f_own) + at, (label, "output fitness", k,
                                                                             fitness[k], f_own)
    return n_ok, n_free


def output_gate(ps, X, y, kind, gpu_cmp, stats: Stats, idx=None, label=""):
    """Runs the output gate on the GPU for the programs `stats` left
    unchecked: gpu_cmp is the fitness array given to check(), idx the
    program index (in ps) of each of its positions (None: the same).
    Returns (programs, cases checked, cases without a bound)."""
    if not stats.unchecked:
        return 0, 0, 0
    import torch
    from paper_2603_12292_amd import api
    prog = [int(idx[i]) if idx is not None else int(i) for i in stats.unchecked]
    sub = ps.subset(prog)
    outs = api.predict(api.DevicePrograms.from_programset(sub), torch.from_numpy(np.ascontiguousarray(X)).cuda())
    outs = outs.cpu().numpy()
    ok, free = check_outputs([ps.program(p) for p in prog], X, y, kind, outs,
                             [float(gpu_cmp[i]) for i in stats.unchecked], label=label)
    return len(prog), ok, free
