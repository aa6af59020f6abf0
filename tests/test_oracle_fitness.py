"""Pins of the oracle's fitness reductions (CPU only)."""
import math
import statistics

import numpy as np
import pytest

from oracle import fitness as fit
from oracle import interp, population
from paper_2603_12292_amd import workloads as wl
from progtext import parse


def test_mse_matches_numpy():
    rng = np.random.default_rng(3)
    yh = rng.standard_normal(1000) * 10
    y = rng.standard_normal(1000).astype(np.float32)
    assert fit.mse(yh, y) == pytest.approx(np.mean((yh - y.astype(np.float64)) ** 2), rel=1e-13)


def test_mse_classification():
    y = np.ones(4, dtype=np.float32)
    assert math.isnan(fit.mse([1, 2, np.nan, np.inf], y))
    assert fit.mse([1, 2, -np.inf, 3], y) == math.inf
    # binary32-scale outputs cannot overflow a binary64 sum
    big = float(np.finfo(np.float32).max)
    assert math.isfinite(fit.mse([big, -big, big, -big], -y))


def test_non_finite_targets():
    """Targets holding invalid values (section 2.1.5 expects such datasets):
    MSE follows IEEE arithmetic of its case terms, 1 - r^2 is undefined."""
    yh = np.array([1.0, 2.0, 3.0, 4.0])
    nan_y = np.array([1, np.nan, 3, 4], dtype=np.float32)
    inf_y = np.array([1, np.inf, 3, 4], dtype=np.float32)
    assert math.isnan(fit.mse(yh, nan_y))
    assert fit.mse(yh, inf_y) == math.inf
    # an infinite output meeting the same infinite target: inf - inf is NaN
    assert math.isnan(fit.mse([1.0, np.inf, 3.0, 4.0], inf_y))
    assert fit.mse([1.0, -np.inf, 3.0, 4.0], inf_y) == math.inf
    # NaN anywhere beats +Inf elsewhere
    assert math.isnan(fit.mse([np.inf, 2.0, 3.0, 4.0], nan_y))
    # 1 - r^2 is NaN, never a perfect 0, for a NaN or infinite target
    rng = np.random.default_rng(6)
    a = rng.standard_normal(50)
    for bad in (np.nan, np.inf, -np.inf):
        y = rng.standard_normal(50).astype(np.float32)
        y[7] = bad
        assert math.isnan(fit.corr_fitness(a, y))
        assert math.isnan(fit.fitness(fit.CORR, a, y))


def test_pearson_matches_library_routines():
    rng = np.random.default_rng(4)
    for _ in range(20):
        x = rng.standard_normal(500) * rng.uniform(0.1, 100) + rng.uniform(-1e3, 1e3)
        y = (0.3 * x + rng.standard_normal(500)).astype(np.float32)
        r = fit.pearson_r(x, y)
        assert r == pytest.approx(statistics.correlation(list(x), [float(v) for v in y]), rel=1e-12)
        assert r == pytest.approx(np.corrcoef(x, y.astype(np.float64))[0, 1], rel=1e-12)
        assert fit.corr_fitness(x, y) == pytest.approx(1 - r * r, rel=1e-12, abs=1e-15)


def test_corr_symmetry_bounds_and_degenerate_cases():
    rng = np.random.default_rng(5)
    a = rng.standard_normal(300).astype(np.float32).astype(np.float64)
    b = rng.standard_normal(300).astype(np.float32)
    assert fit.corr_fitness(a, b) == pytest.approx(fit.corr_fitness(b.astype(np.float64), a.astype(np.float32)), rel=1e-12)
    assert 0.0 <= fit.corr_fitness(a, b) <= 1.0
    assert fit.corr_fitness(np.full(300, 2.5), b) == 1.0          # Sxx == 0 -> r := 0
    assert math.isnan(fit.corr_fitness(a, np.ones(300, dtype=np.float32)))   # Syy == 0
    assert math.isnan(fit.corr_fitness(np.r_[a[:-1], np.inf], b))
    # perfect (anti-)correlation
    assert fit.corr_fitness(-3.0 * b.astype(np.float64) + 7.0, b) == pytest.approx(0.0, abs=1e-14)


def _data(M=2000, D=3, seed=9):
    return wl.make_dataset(seed, M, D, x_range=(1.0, 5.0), target_len=10)


def test_exact_formula_programs():
    """y := the program's own fp32 output -> O32e MSE is exactly 0, r = 1."""
    d = _data()
    rng = np.random.default_rng(11)
    for _ in range(30):
        toks, consts = wl.random_program(rng, int(rng.integers(3, 25)), 3)
        y32 = interp.run(toks, consts, d.X, "o32e")
        if not np.all(np.isfinite(y32)) or np.ptp(y32) == 0:
            continue
        y = y32.astype(np.float32)
        assert fit.mse(y32, y) == 0.0
        f = fit.corr_fitness(y32, y)
        assert f == pytest.approx(0.0, abs=1e-12)
        # and the binary64 MSE is exactly the mean squared fp32 rounding gap
        y64 = interp.run(toks, consts, d.X, "o64")
        gap = y64 - y32
        assert fit.mse(y64, y) == pytest.approx(float(np.mean(gap * gap)), rel=1e-12, abs=1e-300)


def test_affine_invariance_of_correlation_fitness():
    """F(P) == F(P * c_a + c_b) for correlation fitness (O64)."""
    d = _data()
    rng = np.random.default_rng(12)
    checked = 0
    for _ in range(60):
        toks, consts = wl.random_program(rng, int(rng.integers(3, 20)), 3, max_consts=6)
        yh = interp.run(toks, consts, d.X, "o64")
        if not np.all(np.isfinite(yh)) or np.std(yh) < 1e-6 * (np.abs(np.mean(yh)) + 1e-30):
            continue
        na = len(consts)
        t2 = list(toks) + [10 | (na << 8), 2, 10 | ((na + 1) << 8), 0]
        c2 = list(consts) + [-2.5, 1.75]
        f1 = fit.corr_fitness(yh, d.y)
        f2 = fit.corr_fitness(interp.run(t2, c2, d.X, "o64"), d.y)
        assert f2 == pytest.approx(f1, rel=1e-9, abs=1e-12)
        checked += 1
    assert checked > 20


def test_fp32_overflow_classification_differs_from_fp64():
    """e^80 * e^80 * e^80 overflows binary32 but not binary64: O32e +Inf / NaN, O64 finite."""
    X = np.array([[100.0]] * 4, dtype=np.float32)
    toks = parse("x0 exp x0 exp * x0 exp *")
    assert math.isfinite(interp.run(toks, [], X, "o64")[0])
    assert interp.run(toks, [], X, "o32e")[0] == math.inf
    y = np.ones(4, dtype=np.float32)
    f32, _ = population.evaluate_one(toks, [], X, y, fit.MSE, "o32e")
    assert f32 == math.inf
    s = parse("x0 exp x0 exp * x0 exp * sin")
    assert math.isnan(population.evaluate_one(s, [], X, y, fit.MSE, "o32e")[0])
    assert math.isfinite(population.evaluate_one(s, [], X, y, fit.MSE, "o64")[0])


def test_population_pool_equals_serial():
    d = _data(M=500)
    P = wl.random_population(21, 40, 3, 20, 3)
    args = (P.tokens, P.tok_offset, P.tok_len, P.consts, P.const_offset, P.const_count, d.X, d.y)
    for kind in (fit.MSE, fit.CORR):
        f1, s1 = population.evaluate_population(*args, kind)
        f2, s2 = population.evaluate_population(*args, kind, processes=3)
        assert np.array_equal(f1, f2, equal_nan=True) and np.array_equal(s1, s2)


def test_invalid_program_gives_nan_and_status():
    d = _data(M=100)
    f, st = population.evaluate_one(parse("x0 +"), [], d.X, d.y, fit.MSE)
    assert math.isnan(f) and st == interp.ST_UNDERFLOW
