"""Pins of the oracle's Eq. 2 and Eq. 3 scores (CPU only).

Worked values below are computed by hand from the equations; the other pins
are properties the equations fix (symmetry, exact scale invariance, the
affine invariance of r) and a library correlation routine."""
import math

import numpy as np
import pytest

from oracle import scores as sc

NAN, INF = float("nan"), float("inf")


@pytest.mark.parametrize("yh, y, smax, expect", [
    (2.0, 2.0, 1000, 1000),            # ratio 1
    (1.0, 4.0, 1000, 250),             # round(1000 * 1/4)
    (4.0, 1.0, 1000, 250),             # symmetric
    (-1.0, 4.0, 1000, 159),            # round(250 - 90.909...) = round(159.09)
    (3.0, -4.0, 1000, 659),            # round(750 - 90.909...) = round(659.09)
    (0.0, 0.0, 1000, 1000),            # max(|yh|, |y|) = 0
    (0.0, 5.0, 1000, 0),               # ratio 0, product 0: no penalty
    (-0.0, 5.0, 1000, 0),
    (1.0, 4.0, 10, 2),                 # 2.5 rounds half to even -> 2
    (7.0, 20.0, 10, 4),                # 3.5 -> 4
    (-1.0, 2.0, 22, 9),                # 11 - 2 = 9 exactly
    (NAN, NAN, 1000, 1000),            # both invalid
    (INF, NAN, 1000, 1000),
    (-INF, INF, 1000, 1000),
    (1.0, NAN, 1000, -1000),           # one invalid
    (NAN, 0.0, 1000, -1000),
    (INF, 3.0, 1000, -1000),
])
def test_case_score_worked_values(yh, y, smax, expect):
    assert sc.case_score(yh, y, smax) == expect


def test_point_score_sums_cases():
    yh = np.array([2.0, -1.0, NAN, 0.0], dtype=np.float32)
    y = np.array([2.0, 4.0, NAN, 3.0], dtype=np.float32)
    assert sc.point_score(yh, y, 1000) == 1000 + 159 + 1000 + 0


def test_point_score_symmetry_and_scale_invariance():
    rng = np.random.default_rng(5)
    a = rng.normal(0, 10, 500).astype(np.float32)
    b = rng.normal(0, 10, 500).astype(np.float32)
    a[::37] = np.nan
    b[::41] = np.inf
    s = sc.point_score(a, b, 1000)
    assert s == sc.point_score(b, a, 1000)
    # a power-of-two scale of both sides leaves every ratio exact
    assert s == sc.point_score(a * np.float32(8), b * np.float32(8), 1000)
    assert s == sc.point_score(a * np.float32(2 ** -20), b * np.float32(2 ** -20), 1000)
    # every case score lies in [-S, S]
    assert abs(s) <= 1000 * len(a)


def test_valid_pair_r_against_library():
    rng = np.random.default_rng(6)
    a = rng.normal(0, 1, 300)
    b = (0.6 * a + rng.normal(0, 1, 300)).astype(np.float32)
    a[::13] = np.nan
    b[::17] = -np.inf
    keep = np.isfinite(a) & np.isfinite(b)
    r_lib = np.corrcoef(a[keep], b[keep].astype(np.float64))[0, 1]
    assert sc.valid_pair_r(a, b) == pytest.approx(r_lib, rel=1e-12)


def test_r4_score_closed_forms():
    rng = np.random.default_rng(7)
    y = rng.uniform(-5, 5, 200).astype(np.float32)
    # y_hat an affine function of y: |r| = 1, r^4 = 1, score = S N
    yh = 3.0 * y.astype(np.float64) - 2.0
    assert sc.r4_score(yh, y, 50) == pytest.approx(50 * 200, rel=1e-12)
    assert sc.r4_score(-yh, y, 50) == pytest.approx(50 * 200, rel=1e-12)
    # k1 one-invalid and k2 both-invalid pairs: S r^4 (N - k1 - k2) - S (k1 - k2)
    y2 = y.copy()
    yh2 = yh.copy()
    yh2[:7] = np.nan                    # 7 pairs with one invalid
    y2[10:15] = np.nan                  # 5 both invalid
    yh2[10:15] = np.inf
    assert sc.pair_counts(yh2, y2) == (200 - 12, 7, 5)
    assert sc.r4_score(yh2, y2, 50) == pytest.approx(50 * (200 - 12) - 50 * (7 - 5), rel=1e-12)


def test_r4_score_degenerate():
    y = np.array([1.0, 2.0, NAN, 4.0], dtype=np.float32)
    # one valid pair only: r := 0; c1 = 2 (cases 0, 3), c2 = 1 (case 2)
    yh = np.array([NAN, 5.0, INF, NAN])
    assert sc.pair_counts(yh, y) == (1, 2, 1)
    assert sc.r4_score(yh, y, 10) == -10 * (2 - 1)
    # constant output over the valid pairs: r := 0
    yh = np.array([3.0, 3.0, NAN, 3.0])
    assert sc.r4_score(yh, y, 10) == -10 * (0 - 1)
    # r^4 of a partial correlation lies in (0, 1)
    yh = np.array([1.0, 3.0, NAN, 2.0])
    r = sc.valid_pair_r(yh, y)
    assert 0 < r < 1
    assert sc.r4_score(yh, y, 10) == pytest.approx(10 * r ** 4 * 3 + 10, rel=1e-12)
