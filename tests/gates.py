"""Parity gates between GPU fitness and the CPU oracle.

Classification gate: the GPU fitness class (finite / +inf / nan) equals the
class the fp32-emulating oracle (O32e) gives; an fp32 evaluation can
overflow where binary64 does not, so the classes come from O32e, not from
the binary64 oracle.

Value gate: |F_gpu - F_O64| <= 1e-5 |F_O64| + atol for every program that is
finite in both and well conditioned: its fitness moves by at most
1e-6 |F_O64| + atol (a tenth of the gate) when every token is rounded to fp32
(O32e) and in two runs where every sin/cos/exp/log result is also perturbed
by a few ulps (O32p, two seeds) -- a model of an fp32 implementation with
correctly rounded + - * / sqrt and transcendentals accurate to a few ulps,
as the GPU's are.  Ill-conditioned
programs (e.g. sin of exp of a large argument) are counted, not compared.
atol = 1e-10 * mean(y^2) for MSE, 1e-9 for correlation fitness.
"""
import math

import numpy as np

from oracle import fitness as ofit
from oracle import population as opop

RTOL = 1e-5
RTOL_COND = 1e-6


def atol(kind, y):
    y64 = np.asarray(y, dtype=np.float64)
    return 1e-10 * float(np.mean(y64 * y64)) if kind == ofit.MSE else 1e-9


def oracle(ps, X, y, kind, mode, subset=None, processes=None, seed=0):
    return opop.evaluate_population(ps.tokens, ps.tok_offset, ps.tok_len, ps.consts, ps.const_offset,
                                    ps.const_count, X, y, kind, mode, subset=subset, processes=processes,
                                    seed=seed)


def references(ps, X, y, kind, subset=None, processes=None):
    """(F_O64, status, F_O32e, [F_O32p seed 1, seed 2])."""
    f64, s64 = oracle(ps, X, y, kind, "o64", subset, processes)
    f32, _ = oracle(ps, X, y, kind, "o32e", subset, processes)
    pert = [oracle(ps, X, y, kind, "o32p", subset, processes, seed=s)[0] for s in (1, 2)]
    return f64, s64, f32, pert


def check(gpu, f64, f32e, kind, y, max_ill_frac=0.05, label="", perturbed=()):
    """Apply both gates; returns (n_compared, n_ill)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    at = atol(kind, y)
    cls_gpu = [ofit.classify(v) for v in gpu]
    cls_32 = [ofit.classify(v) for v in f32e]
    bad_cls = [i for i in range(len(gpu)) if cls_gpu[i] != cls_32[i]]
    assert not bad_cls, (label, "classification", [(i, gpu[i], f32e[i], f64[i]) for i in bad_cls[:10]])
    n_cmp = n_ill = 0
    bad = []
    for i in range(len(gpu)):
        if not (math.isfinite(gpu[i]) and math.isfinite(f64[i]) and math.isfinite(f32e[i])):
            continue
        spread = max([abs(f32e[i] - f64[i])] + [abs(p[i] - f64[i]) for p in perturbed])
        if not all(math.isfinite(p[i]) for p in perturbed) or spread > RTOL_COND * abs(f64[i]) + at:
            n_ill += 1
            continue
        n_cmp += 1
        if abs(gpu[i] - f64[i]) > RTOL * abs(f64[i]) + at:
            bad.append((i, gpu[i], f64[i], f32e[i]))
    assert not bad, (label, "value", bad[:10])
    finite = sum(1 for c in cls_32 if c == "finite")
    assert n_ill <= max_ill_frac * max(finite, 1) + 2, (label, "too many ill-conditioned", n_ill, finite)
    return n_cmp, n_ill
