"""Pins of the oracle's first-order fitness bound (oracle/bound.py), CPU only.

The bound B is pinned three ways:
  * closed forms worked by hand for small programs;
  * an independent evaluator (the recursive tree evaluator, scalar Python)
    run with the worst-case errors the bound assumes imposed on each
    operation: the fitness must move by B to first order (a wrong partial
    derivative, a wrong sign or a dropped term makes it move by less or by
    more), and by at most B under random errors of the same size;
  * the fp32-emulating oracle with perturbed transcendentals (o32p) stays
    within the bound of o32e on a whole workload, which is the use the
    parity gate makes of it.
"""
import math

import numpy as np
import pytest

from oracle import bound as ob
from oracle import fitness as ofit
from oracle import interp, tree
from paper_2603_12292_amd import workloads as wl
from progtext import parse

ULP = 2.0 ** -23
TINY = 2.0 ** -149


def _r32(v):
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def _data(M=500, D=3, seed=41, lo=1.0, hi=4.0):
    return wl.make_dataset(seed, M, D, x_range=(lo, hi), target_len=8)


def test_token_eps_rules():
    # x0 x1 + : nothing approximate, nothing tainted
    toks = parse("x0 x1 +")
    _, ch = ob.tape(toks, [], np.ones((2, 2), np.float32))
    assert ob.token_eps(toks, ch)[0] == [0.0, 0.0, 0.0]
    # x0 sin x1 + c0 * : sin 4 ulp, + and * tainted (1 ulp), terminals 0
    toks = parse("x0 sin x1 + c0 *")
    _, ch = ob.tape(toks, [1.0], np.ones((2, 2), np.float32))
    assert ob.token_eps(toks, ch)[0] == [0.0, 4 * ULP, 0.0, ULP, 0.0, ULP]
    # sqrt is faithful (2 ulp budget); a division of untainted operands is exact,
    # unless the implementation's division is not correctly rounded
    toks = parse("x0 x1 / sqrt")
    _, ch = ob.tape(toks, [], np.ones((2, 2), np.float32))
    assert ob.token_eps(toks, ch)[0] == [0.0, 0.0, 0.0, 2 * ULP]
    assert ob.token_eps(toks, ch, div_eps=2 * ULP)[0] == [0.0, 0.0, 2 * ULP, 2 * ULP]
    # the library functions of the further operators: 8 ulp
    toks = parse("x0 atan")
    _, ch = ob.tape(toks, [], np.ones((2, 1), np.float32))
    assert ob.token_eps(toks, ch)[0] == [0.0, 8 * ULP]


def test_closed_form_exp_mse():
    d = _data()
    x = d.X[:, 0].astype(np.float64)
    y = d.y.astype(np.float64)
    M = len(y)
    v = _r32(np.exp(x))  # o32e value of exp(x0)
    a = np.abs(2.0 * (v - y) / M)
    expect = math.fsum((a * (v * 4 * ULP + TINY)).tolist())
    got = ob.fitness_bound(parse("x0 exp"), [], d.X, d.y, ofit.MSE)
    assert got == pytest.approx(expect, rel=1e-12)


def test_closed_form_sin_times_x_mse():
    d = _data()
    x0 = d.X[:, 0].astype(np.float64)
    x1 = d.X[:, 1].astype(np.float64)
    y = d.y.astype(np.float64)
    M = len(y)
    s = _r32(np.sin(x0))
    yh = _r32(s * x1)
    a_top = np.abs(2.0 * (yh - y) / M)
    # the product (tainted, 1 ulp) and the sine (4 ulp, adjoint a_top * x1)
    expect = math.fsum((a_top * (np.abs(yh) * ULP + TINY)).tolist()) + \
        math.fsum((a_top * x1 * (np.abs(s) * 4 * ULP + TINY)).tolist())
    got = ob.fitness_bound(parse("x0 sin x1 *"), [], d.X, d.y, ofit.MSE)
    assert got == pytest.approx(expect, rel=1e-12)


def test_closed_form_corr_scale():
    # F(c * exp(x0)) under 1 - r^2: only the exp token carries error, and
    # the product with an exact constant is tainted; the adjoint of exp's
    # output is c * dF/dyhat
    d = _data()
    x = d.X[:, 0].astype(np.float64)
    c = float(np.float32(2.5))
    e = _r32(np.exp(x))
    yh = _r32(c * e)
    F, sd = ob.seed(ofit.CORR, yh, d.y)
    assert F == pytest.approx(ofit.corr_fitness(yh, d.y), rel=0, abs=0)
    expect = math.fsum((np.abs(sd) * (np.abs(yh) * ULP + TINY)).tolist()) + \
        math.fsum((np.abs(sd * c) * (e * 4 * ULP + TINY)).tolist())
    got = ob.fitness_bound(parse("x0 exp c0 *"), [2.5], d.X, d.y, ofit.CORR)
    assert got == pytest.approx(expect, rel=1e-12)


def test_exact_programs_have_zero_bound():
    d = _data()
    for prog, consts in (("x0 x1 + c0 *", [1.5]), ("x0 x1 / x2 -", []), ("x0 x0 - x1 /", []),
                         ("c0 x1 * x2 x0 / +", [0.25])):
        assert ob.fitness_bound(parse(prog), consts, d.X, d.y, ofit.MSE) == 0.0
        assert ob.fitness_bound(parse(prog), consts, d.X, d.y, ofit.CORR) == 0.0


def test_branch_points():
    d = _data()
    # an untainted zero at log's branch point stays there: the log token
    # contributes its tiny term only (value 0), the sum above it (tainted by
    # the approximate log) its 1-ulp term
    b = ob.fitness_bound(parse("x0 x0 - log x1 +"), [], d.X, d.y, ofit.MSE)
    yh = d.X[:, 1].astype(np.float64)
    a = np.abs(2.0 * (yh - d.y.astype(np.float64)) / len(yh))
    assert b == pytest.approx(math.fsum((a * (yh * ULP + TINY)).tolist()) + math.fsum((a * TINY).tolist()),
                              rel=1e-12)
    # a tainted zero may move off it: no first-order bound
    assert ob.fitness_bound(parse("x0 sin x0 sin - log x1 +"), [], d.X, d.y, ofit.MSE) == math.inf
    assert ob.fitness_bound(parse("x1 x0 sin x0 sin - /"), [], d.X, d.y, ofit.MSE) == math.inf
    assert ob.fitness_bound(parse("x0 sin x0 sin - sqrt x1 +"), [], d.X, d.y, ofit.MSE) == math.inf
    # a non-finite fitness has no bound
    assert math.isnan(ob.fitness_bound(parse("x0 x0 - c0 /"), [0.0], d.X, d.y, ofit.MSE)) is False
    X = np.full((20, 1), 100.0, dtype=np.float32)
    yy = np.linspace(0, 1, 20).astype(np.float32)
    assert math.isnan(ob.fitness_bound(parse("x0 exp x0 exp * x0 exp *"), [], X, yy, ofit.MSE))


def _smooth_programs(n, D, seed):
    """Random programs over the nine operators whose outputs stay finite and
    away from branch points on X in [1, 3]."""
    rng = np.random.default_rng(seed)
    X = np.random.default_rng(seed + 1).uniform(1.0, 3.0, (30, D)).astype(np.float32)
    out = []
    while len(out) < n:
        toks, consts = wl.random_program(rng, int(rng.integers(3, 24)), D)
        yh = interp.run(toks, consts, X, "o64")
        if not np.all(np.isfinite(yh)) or np.ptp(yh) == 0.0 or np.max(np.abs(yh)) > 1e6:
            continue
        out.append((toks, consts))
    return out, X


@pytest.mark.parametrize("kind", [ofit.MSE, ofit.CORR])
def test_worst_case_errors_move_fitness_by_the_bound(kind):
    """Imposing d[t,i] = eps[t] sign(A[t,i] v[t,i]) on every operation through
    the independent tree evaluator moves the fitness by B (first order; the
    errors are scaled down to 2^-10 of their budgets to stay linear);
    random errors of the same size move it by at most B."""
    progs, X = _smooth_programs(40, 2, 7)
    y = np.random.default_rng(3).normal(2.0, 1.0, X.shape[0]).astype(np.float32)
    scale = 2.0 ** -10
    rng = np.random.default_rng(11)
    checked = 0
    for toks, consts in progs:
        B = ob.fitness_bound(toks, consts, X, y, kind, base="o64", eps_scale=scale)
        F0 = ofit.fitness(kind, interp.run(toks, consts, X, "o64"), y)
        if not math.isfinite(B) or B > 1e-6 * max(abs(F0), 1e-3):
            # errors of relative size 2^-31 moving F by more than 1e-6 of it:
            # an intermediate value is within the perturbation of a zero or a
            # pole (e.g. log|log x| near x = 1), the first-order regime is left
            continue
        values, children = ob.tape(toks, consts, X, "o64")
        _, sd = ob.seed(kind, values[-1], y)
        eps, tainted = ob.token_eps(toks, children, eps_scale=scale)
        adj = ob.adjoints(toks, values, children, sd, tainted)
        base = tree.run(toks, consts, X)
        assert np.array_equal(base, values[-1])
        sign = {t: np.sign(adj[t] * values[t]) for t in range(len(toks)) if eps[t] > 0.0}
        worst = tree.run(toks, consts, X,
                         perturb=lambda pos, row, v: v * (1.0 + eps[pos] * sign[pos][row]) if pos in sign else v)
        dF = ofit.fitness(kind, worst, y) - F0
        if B < 1e-12 * max(abs(F0), 1e-3):
            continue  # below what binary64 resolves
        assert dF == pytest.approx(B, rel=2e-3), (toks, B, dF)
        for _ in range(2):
            rnd = {t: rng.uniform(-1.0, 1.0, X.shape[0]) for t in sign}
            pert = tree.run(toks, consts, X,
                            perturb=lambda pos, row, v: v * (1.0 + eps[pos] * rnd[pos][row]) if pos in rnd else v)
            assert abs(ofit.fitness(kind, pert, y) - F0) <= B * (1 + 2e-3)
        checked += 1
    assert checked >= 25


@pytest.mark.parametrize("kind", [ofit.MSE, ofit.CORR])
def test_o32p_within_bound_on_tiny_workload(kind):
    """The fp32-emulating oracle with perturbed approximate operators (o32p:
    up to 2^-22 relative, then rounded: within the 4-ulp budget) stays within
    twice the bound of o32e on every finite program of the tiny workload --
    the envelope the GPU parity gate applies."""
    w = wl.config_tiny()
    ps = w.programs
    n_fin = n_inf = 0
    for p in range(ps.n):
        o, l = int(ps.tok_offset[p]), int(ps.tok_len[p])
        co, cc = int(ps.const_offset[p]), int(ps.const_count[p])
        toks, consts = ps.tokens[o:o + l], ps.consts[co:co + cc]
        yh = interp.run(toks, consts, w.data.X, "o32e")
        f32 = ofit.fitness(kind, yh, w.data.y)
        if not math.isfinite(f32) or (kind == ofit.CORR and np.all(yh == yh[0])):
            # (o32p draws its perturbations per case, so it turns a program
            # without variables into a varying one, which no evaluation does)
            continue
        B = ob.fitness_bound(toks, consts, w.data.X, w.data.y, kind)
        if B == math.inf:
            n_inf += 1
            continue
        for s in (1, 2):
            fp = ofit.fitness(kind, interp.run(toks, consts, w.data.X, "o32p", seed=s), w.data.y)
            assert abs(fp - f32) <= 2.0 * B + 1e-12 * abs(f32), (p, f32, fp, B)
        n_fin += 1
    assert n_fin > 150 and n_inf <= 0.05 * n_fin, (n_fin, n_inf)
