"""The paper's own fitness scores in float64 -- test infrastructure.

Section 2.1.5 of the paper defines two scores, both maximised, that pair
invalid values (NaN, +Inf, -Inf) in the model output with invalid values in
the target instead of discarding them.  S is the maximum score parameter.

Point-to-point score (Eq. 3), per case i:
  both valid:   S                                  if max(|y_hat|, |y|) == 0
                round(S min/max - S/11)            if y_hat y < 0
                round(S min/max)                   otherwise
                (min/max of |y_hat_i|, |y_i|)
  both invalid: S        (agreement rewarded)
  one invalid:  -S       (disagreement penalised)
and the program's score aggregates the case scores.

Correlation score (Eq. 2): with c1 the number of cases where exactly one of
y_hat_i, y_i is invalid and c2 the number where both are, and r Pearson's
coefficient (Eq. 1) over the cases where both are valid,
  score = S r^4 (N - (c1 + c2)) - S (c1 - c2).

Readings where the paper is silent:
  * the case scores are aggregated by summation;
  * round() rounds half to even, applied to the binary64 value of
    S * (min / max) - S / 11 (S / 11 real-valued), min / max computed in
    binary64 from the binary32 values;
  * y_hat y < 0 means nonzero values of opposite signs (decided exactly);
  * r is computed by the two-pass centred definition over the valid pairs;
    r := 0 when fewer than two pairs are valid or either side has zero
    variance over them.
Every value here is a plain loop or an exactly rounded sum (math.fsum).
"""
from __future__ import annotations

import math

import numpy as np


def _valid(v: float) -> bool:
    return math.isfinite(v)


def case_score(yh: float, y: float, smax: float) -> float:
    """Eq. 3 for one case (binary64 arithmetic on the given values)."""
    vh, vy = _valid(yh), _valid(y)
    if not vh and not vy:
        return float(smax)
    if vh != vy:
        return -float(smax)
    a, b = abs(yh), abs(y)
    hi, lo = max(a, b), min(a, b)
    if hi == 0.0:
        return float(smax)
    t = smax * (lo / hi)
    if (yh < 0.0 < y) or (y < 0.0 < yh):
        t = t - smax / 11.0
    return float(round(t))  # Python's round(): half to even


def point_score(y_hat, y, smax: float) -> float:
    """Sum over cases of Eq. 3."""
    yh = np.asarray(y_hat, dtype=np.float64)
    yt = np.asarray(y, dtype=np.float32).astype(np.float64)
    return math.fsum(case_score(float(a), float(b), smax) for a, b in zip(yh.tolist(), yt.tolist()))


def pair_counts(y_hat, y):
    """(n_valid_pairs, c1, c2) of Eq. 2."""
    yh = np.asarray(y_hat, dtype=np.float64)
    yt = np.asarray(y, dtype=np.float32).astype(np.float64)
    n = c1 = c2 = 0
    for a, b in zip(yh.tolist(), yt.tolist()):
        va, vb = _valid(a), _valid(b)
        if va and vb:
            n += 1
        elif va or vb:
            c1 += 1
        else:
            c2 += 1
    return n, c1, c2


def valid_pair_r(y_hat, y) -> float:
    """Eq. 1 over the pairs where both values are valid (0 when degenerate)."""
    yh = np.asarray(y_hat, dtype=np.float64)
    yt = np.asarray(y, dtype=np.float32).astype(np.float64)
    keep = np.isfinite(yh) & np.isfinite(yt)
    a, b = yh[keep], yt[keep]
    n = a.shape[0]
    if n < 2:
        return 0.0
    ma = math.fsum(a.tolist()) / n
    mb = math.fsum(b.tolist()) / n
    u, w = a - ma, b - mb
    sxx = math.fsum((u * u).tolist())
    syy = math.fsum((w * w).tolist())
    if sxx == 0.0 or syy == 0.0:
        return 0.0
    return math.fsum((u * w).tolist()) / math.sqrt(sxx * syy)


def r4_score(y_hat, y, smax: float) -> float:
    """Eq. 2."""
    n, c1, c2 = pair_counts(y_hat, y)
    N = n + c1 + c2
    r = valid_pair_r(y_hat, y)
    return smax * r ** 4 * (N - (c1 + c2)) - smax * (c1 - c2)
