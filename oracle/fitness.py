"""Fitness reductions in float64 -- test infrastructure.

Section 2.1.5 of the paper: a point-to-point fitness compares the model
output y_hat with the target y case by case and aggregates; the correlation
fitness starts from Pearson's r (Eq. 1), and the 1 - r^2 objective (named in
the same section as the one earlier work minimised) is the correlation
fitness the library computes.  The point-to-point fitness here is the mean
squared error.

Conventions where the paper is silent (it pairs invalid values instead):
  MSE   the case terms d_i = y_hat_i - y_i in IEEE binary64: any NaN d_i
        (a NaN output or target, or an infinite output equal to an infinite
        target) -> NaN; else any +-Inf d_i -> +Inf; else
        (1/M) * sum d_i^2.  For finite targets: any NaN y_hat -> NaN, else
        any +-Inf y_hat -> +Inf.
  CORR  any non-finite y_hat or y -> NaN (Eq. 1's sums are undefined; the
        section 2.1.5 datasets may hold invalid targets); two-pass centred sums
        Sxx = sum (y_hat - mean y_hat)^2, Syy = sum (y - mean y)^2,
        Sxy = sum (y_hat - mean y_hat)(y - mean y);
        Sxx == 0 -> r := 0 (F = 1); Syy == 0 -> NaN;
        else r = Sxy / sqrt(Sxx * Syy), F = min(1, max(0, 1 - r*r)).
Sums use math.fsum (exactly rounded).
"""
from __future__ import annotations

import math

import numpy as np

MSE = 0
CORR = 1


def mse(y_hat, y) -> float:
    yh = np.asarray(y_hat, dtype=np.float64)
    yt = np.asarray(y, dtype=np.float32).astype(np.float64)
    with np.errstate(invalid="ignore"):
        d = yh - yt
    if np.any(np.isnan(d)):
        return math.nan
    if np.any(np.isinf(d)):
        return math.inf
    return math.fsum((d * d).tolist()) / yh.shape[0]


def pearson_sums(y_hat, y):
    """(Sxx, Syy, Sxy) by the two-pass centred definition (Eq. 1's terms)."""
    yh = np.asarray(y_hat, dtype=np.float64)
    yt = np.asarray(y, dtype=np.float32).astype(np.float64)
    M = yh.shape[0]
    mx = math.fsum(yh.tolist()) / M
    my = math.fsum(yt.tolist()) / M
    u = yh - mx
    w = yt - my
    return (math.fsum((u * u).tolist()), math.fsum((w * w).tolist()), math.fsum((u * w).tolist()))


def pearson_r(y_hat, y) -> float:
    """Eq. 1 of the paper (NaN where undefined)."""
    sxx, syy, sxy = pearson_sums(y_hat, y)
    if sxx == 0.0 or syy == 0.0:
        return math.nan
    return sxy / math.sqrt(sxx * syy)


def corr_fitness(y_hat, y) -> float:
    """1 - r^2 with the degenerate-case conventions above."""
    yh = np.asarray(y_hat, dtype=np.float64)
    if not np.all(np.isfinite(yh)) or not np.all(np.isfinite(np.asarray(y, dtype=np.float64))):
        return math.nan
    sxx, syy, sxy = pearson_sums(yh, y)
    if syy == 0.0:
        return math.nan
    if sxx == 0.0:
        return 1.0
    r = sxy / math.sqrt(sxx * syy)
    return min(1.0, max(0.0, 1.0 - r * r))


def fitness(kind: int, y_hat, y) -> float:
    if kind == MSE:
        return mse(y_hat, y)
    if kind == CORR:
        return corr_fitness(y_hat, y)
    raise ValueError(kind)


def classify(f: float) -> str:
    """Fitness class used by the classification gate: finite, +inf or nan."""
    if math.isnan(f):
        return "nan"
    if math.isinf(f):
        return "+inf" if f > 0 else "-inf"
    return "finite"
