"""Pins of the oracle's fitness bound (oracle/bound.py), CPU only.

The bound B is pinned four ways:
  * closed forms worked by hand for small programs;
  * brute force for the fitness combinations: with every output moved by at
    most b[i], the largest change of the MSE or of 1 - r^2 over every corner
    of that box (the extreme of a function this close to linear lies at a
    corner) is at most B, and B is not much larger;
  * an independent evaluator (the recursive tree evaluator, scalar Python)
    run with the worst-case errors imposed on each operation (signs from
    the reverse-mode adjoints): the fitness moves by B to first order (a
    wrong bound rule, a wrong sign or a dropped term makes it move by less
    or more), and by at most B under random errors of the same size;
  * the fp32-emulating oracle with perturbed functions (o32p) stays within
    the bound of o32e on a whole workload, the use the parity gate makes.
"""
import itertools
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


def _mse_of(yh, y, b):
    d = np.abs(yh - y.astype(np.float64))
    return math.fsum((2 * d * b + b * b).tolist()) / len(yh)


def test_token_eps_rules():
    eps, always = ob.token_eps(parse("x0 sin x1 + c0 * sqrt"))
    assert eps == [0.0, 4 * ULP, 0.0, ULP, 0.0, ULP, 2 * ULP]
    assert always == [False, True, False, False, False, False, True]
    eps, always = ob.token_eps(parse("x0 x1 /"), div_eps=2 * ULP)
    assert eps == [0.0, 0.0, 2 * ULP] and always == [False, False, True]
    assert ob.token_eps(parse("x0 atan"))[0] == [0.0, 8 * ULP]
    # correctly rounded operators on exact operands carry no error
    d = _data()
    _, _, dd, rel = ob.case_bounds(parse("x0 x1 + x2 * c0 /"), [0.75], d.X)
    assert all(np.all(v == 0.0) for v in dd) and all(np.all(r == 0.0) for r in rel)


def test_closed_form_exp_mse():
    d = _data()
    x = d.X[:, 0].astype(np.float64)
    v = _r32(np.exp(x))              # o32e value of exp(x0)
    b = 4 * ULP * v + TINY           # exact operand: only exp's own error
    got = ob.fitness_bound(parse("x0 exp"), [], d.X, d.y, ofit.MSE)
    assert got == pytest.approx(_mse_of(v, d.y, b), rel=1e-12)


def test_closed_form_sin_times_x_mse():
    d = _data()
    x0 = d.X[:, 0].astype(np.float64)
    x1 = d.X[:, 1].astype(np.float64)
    s = _r32(np.sin(x0))
    yh = _r32(s * x1)
    ds = 4 * ULP * np.abs(s) + TINY          # the sine's own error
    p = np.abs(x1) * ds                      # carried through the product
    b = p + ULP * (np.abs(yh) + p) + TINY    # the product re-rounds an inexact operand
    got = ob.fitness_bound(parse("x0 sin x1 *"), [], d.X, d.y, ofit.MSE)
    assert got == pytest.approx(_mse_of(yh, d.y, b), rel=1e-12)


def test_closed_form_division_and_log():
    d = _data()
    x0 = d.X[:, 0].astype(np.float64)
    x1 = d.X[:, 1].astype(np.float64)
    # x1 / log(x0): log's own error e = 4 ulp |l| + tiny, then the quotient
    # moves by at most |x1| e / (|l| (|l| - e)) and re-rounds
    l = _r32(np.log(x0))
    yh = _r32(x1 / l)
    e = 4 * ULP * np.abs(l) + TINY
    p = np.abs(x1) * e / (np.abs(l) * (np.abs(l) - e))
    b = p + ULP * (np.abs(yh) + p) + TINY
    got = ob.fitness_bound(parse("x1 x0 log /"), [], d.X, d.y, ofit.MSE)
    assert got == pytest.approx(_mse_of(yh, d.y, b), rel=1e-12)


def test_exact_programs_have_zero_bound():
    d = _data()
    for prog, consts in (("x0 x1 + c0 *", [1.5]), ("x0 x1 / x2 -", []), ("x0 x0 - x1 /", []),
                         ("c0 x1 * x2 x0 / +", [0.25])):
        assert ob.fitness_bound(parse(prog), consts, d.X, d.y, ofit.MSE) == 0.0
        assert ob.fitness_bound(parse(prog), consts, d.X, d.y, ofit.CORR) == 0.0


def test_branch_points():
    d = _data()
    # an exact zero at log's branch point stays there: log's own tiny error,
    # then the sum re-rounds an inexact operand
    b = ob.fitness_bound(parse("x0 x0 - log x1 +"), [], d.X, d.y, ofit.MSE)
    x1 = d.X[:, 1].astype(np.float64)
    bb = TINY + ULP * (x1 + TINY) + TINY
    assert b == pytest.approx(_mse_of(x1, d.y, bb), rel=1e-12)
    # an inexact zero may move off it: no bound
    assert ob.fitness_bound(parse("x0 sin x0 sin - log x1 +"), [], d.X, d.y, ofit.MSE) == math.inf
    assert ob.fitness_bound(parse("x1 x0 sin x0 sin - /"), [], d.X, d.y, ofit.MSE) == math.inf
    # the square root is continuous at 0: sqrt of an inexact zero moves by
    # at most the square root of its operand's bound
    bs = ob.fitness_bound(parse("x0 sin x0 sin - sqrt x1 +"), [], d.X, d.y, ofit.MSE)
    assert 0.0 < bs < math.inf
    # a constant output under 1 - r^2: bounded (0) when the outputs stay equal
    assert ob.fitness_bound(parse("c0 sin x0 x0 - +"), [1.25], d.X, d.y, ofit.CORR) == 0.0
    # a non-finite fitness has no bound
    X = np.full((20, 1), 100.0, dtype=np.float32)
    yy = np.linspace(0, 1, 20).astype(np.float32)
    assert math.isnan(ob.fitness_bound(parse("x0 exp x0 exp * x0 exp *"), [], X, yy, ofit.MSE))


@pytest.mark.parametrize("kind", [ofit.MSE, ofit.CORR])
def test_combinations_against_box_corners(kind):
    """The fitness change over every corner of the box |h_i| <= b_i (M = 8):
    never above the bound, and the bound within a few percent of it."""
    rng = np.random.default_rng(7)
    for trial in range(30):
        M = 8
        yh = rng.normal(0.0, 1.0, M) * 10 ** rng.uniform(-1, 2)
        y = rng.normal(0.5, 1.0, M).astype(np.float32)
        yc = y.astype(np.float64) - y.astype(np.float64).mean()
        if trial % 3 == 0:
            yh = y.astype(np.float64) * 2.0 + rng.normal(0.0, 1e-3, M)   # r near 1
        if trial % 3 == 1:
            yh = yh - (yh @ yc) / (yc @ yc) * yc                          # r near 0
        b = np.abs(yh) * rng.uniform(0, 1e-5, M) + 1e-9
        F0 = ofit.fitness(kind, yh, y)
        worst = 0.0
        for signs in itertools.product((-1.0, 1.0), repeat=M):
            worst = max(worst, abs(ofit.fitness(kind, yh + np.array(signs) * b, y) - F0))
        B = ob.mse_bound(yh, y, b) if kind == ofit.MSE else ob.corr_bound(yh, y, b)
        assert worst <= B * (1 + 1e-9) + 1e-15, (trial, worst, B)
        assert B <= 1.05 * worst + 1e-12, (trial, worst, B)


def _smooth_programs(n, D, seed):
    """Random programs over the nine operators whose outputs stay finite on
    X in [1, 3]."""
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
    """Imposing on every operation the error rel[t,i] * sign(A[t,i] v[t,i])
    (budgets scaled to 2^-10 of their size, to stay in the first-order
    regime) through the independent tree evaluator moves the fitness by B
    to first order; random errors of the same size move it by at most B."""
    progs, X = _smooth_programs(40, 2, 7)
    y = np.random.default_rng(3).normal(2.0, 1.0, X.shape[0]).astype(np.float32)
    scale = 2.0 ** -10
    rng = np.random.default_rng(11)
    checked = 0
    for toks, consts in progs:
        B = ob.fitness_bound(toks, consts, X, y, kind, base="o64", eps_scale=scale)
        F0 = ofit.fitness(kind, interp.run(toks, consts, X, "o64"), y)
        if not math.isfinite(B) or B > 1e-6 * max(abs(F0), 1e-3) or B < 1e-12 * max(abs(F0), 1e-3):
            # a value within its error of a zero or pole (first-order regime
            # left), or a change below what binary64 resolves
            continue
        values, children, _, rel = ob.case_bounds(toks, consts, X, "o64", eps_scale=scale)
        _, sd = ob.seed(kind, values[-1], y)
        adj = ob.adjoints(toks, values, children, sd)
        base = tree.run(toks, consts, X)
        assert np.array_equal(base, values[-1])
        sign = {t: np.sign(adj[t] * values[t]) for t in range(len(toks)) if np.any(rel[t] > 0.0)}
        worst = tree.run(toks, consts, X,
                         perturb=lambda pos, row, v: v * (1.0 + rel[pos][row] * sign[pos][row]) if pos in sign else v)
        dF = ofit.fitness(kind, worst, y) - F0
        assert dF == pytest.approx(B, rel=2e-3), (toks, B, dF)
        for _ in range(2):
            rnd = {t: rng.uniform(-1.0, 1.0, X.shape[0]) for t in sign}
            pert = tree.run(toks, consts, X,
                            perturb=lambda pos, row, v: v * (1.0 + rel[pos][row] * rnd[pos][row]) if pos in rnd else v)
            assert abs(ofit.fitness(kind, pert, y) - F0) <= B
        checked += 1
    assert checked >= 25


@pytest.mark.parametrize("kind", [ofit.MSE, ofit.CORR])
def test_o32p_within_bound_on_tiny_workload(kind):
    """The fp32-emulating oracle with perturbed approximate operators (o32p:
    up to 2^-22 relative, then rounded) stays within the bound of o32e
    computed with budgets doubled (which covers those perturbations, the
    square root's included) on every finite program of the tiny workload."""
    w = wl.config_tiny()
    ps = w.programs
    n_fin = n_inf = 0
    for p in range(ps.n):
        toks, consts = ps.program(p)
        yh = interp.run(toks, consts, w.data.X, "o32e")
        f32 = ofit.fitness(kind, yh, w.data.y)
        if not math.isfinite(f32) or (kind == ofit.CORR and np.all(yh == yh[0])):
            # (o32p draws its perturbations per case, so it turns a program
            # without variables into a varying one, which no evaluation does)
            continue
        B = ob.fitness_bound(toks, consts, w.data.X, w.data.y, kind, eps_scale=2.0)
        if B == math.inf:
            n_inf += 1
            continue
        for s in (1, 2):
            fp = ofit.fitness(kind, interp.run(toks, consts, w.data.X, "o32p", seed=s), w.data.y)
            assert abs(fp - f32) <= B * (1 + 1e-9) + 1e-12 * abs(f32), (p, f32, fp, B)
        n_fin += 1
    assert n_fin > 150 and n_inf <= 0.05 * n_fin, (n_fin, n_inf)
