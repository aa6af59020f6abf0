"""Bound on the fitness change of a binary32 evaluation -- test infrastructure.

Why it exists.  The parity claim of the library is a binary32 evaluation per
case (paper, section 2.1.2: every genome is run on every fitness case) whose
+ - * / are correctly rounded and whose other operators are accurate to a
few ulps.  Such an evaluation reproduces the fp32-emulating oracle (mode
"o32e" of ``oracle.interp``) token by token, except that each token's result
may carry a small error of its own, which later tokens carry on.  How far
that moves a program's fitness depends on the program: sin or exp of a
large argument, or a division by a value near zero, amplify it enormously.
This module computes, for one program, a bound B on that movement, so that
every program can be value-checked against the oracle, the ill-conditioned
ones included, with an envelope that follows from the stated operator
accuracies rather than from a tolerance chosen by hand.

Model.  Token t on case i has the value v[t,i] along the base trajectory
(the o32e values by default).  The evaluation under test computes
v'[t,i] = f_t(operands') (1 + e) + (tiny), |e| <= eps[t]: the exact operator
on its own (perturbed) operands, then its own error.

Per-case bound (a running error bound, forward over the postfix tape; the
interval arithmetic of the operators' ranges, in binary64): d[t,i] >=
|v'[t,i] - v[t,i]| follows from the operands' bounds by the operator's
modulus of continuity,
  ADD, SUB   da + db
  MUL        |b| da + |a| db + da db
  DIV        (|b| da + |a| db) / (|b| (|b| - db))        needs db < |b|
  SIN, COS   min(|cos x| dx + dx^2/2, 2) (|sin x| for COS; Taylor's bound)
  EXP        exp(clamp(x + dx)) - exp(clamp(x - dx)) at most, one-sided
  LOG        log(|x| / (|x| - dx))                       needs dx < |x|
  SQRT       the larger of sqrt(|x| + dx) - sqrt|x| and sqrt|x| - sqrt(max(|x| - dx, 0))
  SQUARE     2 |x| dx + dx^2
  RECIP      dx / (|x| (|x| - dx))                       needs dx < |x|
  TAN        dx (1 + max tan^2 at x -+ dx)               needs no pole within dx
  ASIN, ACOS dx / sqrt(1 - (|x| + dx)^2)                 needs |x| + dx < 1
  ATAN, TANH min(dx, pi), min(dx, 2) (1-Lipschitz)
plus the token's own error eps[t] (|v| + d) + 2^-149 (subnormal spacing)
where eps[t] > 0.  A protected operator at its branch point with an exact
operand (DIV with b == 0 and db == 0, LOG with x == 0 and dx == 0) stays on
its branch (bound 0 from there); where a "needs" condition fails, the case
is unbounded (+inf) and so is the program's B ("vacuous": no bound exists).

eps per token (``token_eps``), for a binary32 evaluation against o32e:
  * VAR, CONST: 0 (the same binary32 inputs).
  * SIN COS EXP LOG and the five further library functions: their stated
    accuracy plus o32e's own half ulp, as a relative bound (``EPS_APPROX``).
  * SQRT: faithful (within 1 ulp of the exact value, o32e within 1/2): 2^-22.
  * ADD SUB MUL DIV SQUARE RECIP (correctly rounded): on a case where both
    operands are exact (bound 0), the same rounding of the same value: 0;
    otherwise the two roundings can differ by up to 1 ulp: 2^-23.
    ``div_eps`` sets DIV's for an implementation whose division is not
    correctly rounded.

Fitness bound from the per-case output bounds b[i] (exact, not linearised):
  MSE   |(d + h)^2 - d^2| <= 2 |d| b + b^2 per case, d = yhat - y:
        B = sum_i (2 |d_i| b_i + b_i^2) / M.
  CORR  with s = sqrt(Sxx), g = ||b||_2 and B1 = sum_i |dr/dyhat_i| b_i
        (dr/dyhat_i = w_i / sqrt(Sxx Syy) - r u_i / Sxx, the centred sums of
        Eq. 1), the perturbed r differs from r by at most
            Br = (s B1 + |r| g^2 / (2 (s - g))) / (s - g)      (needs g < s)
        (the centred output u moves by a vector of norm <= g; the norm of
        u is convex with curvature <= 1/(s - g) on that ball), and
        F = 1 - r^2 by at most B = min(Br (2|r| + Br), 1).  A constant
        output (F = 1 by convention): B = 0 when every token carrying error
        has one value on all cases (the outputs stay equal), else +inf.
B is first-order tight: as the errors shrink it approaches the largest
first-order change, sum |dF/dv[t,i]| |v[t,i]| eps[t] over the worst signs
(``adjoints`` gives those derivatives by reverse mode -- Linnainmaa, BIT 16
(1976), introduced reverse accumulation for this estimate of accumulated
rounding error -- and the tests impose exactly those errors).
"""
from __future__ import annotations

import math

import numpy as np

from . import fitness as ofit
from . import interp

ADD, SUB, MUL, DIV, SIN, COS, EXP, LOG, SQRT, VAR, CONST = range(11)
SQUARE, RECIP, TAN, ASIN, ACOS, ATAN, TANH = range(11, 18)

ULP = 2.0 ** -23          # one binary32 ulp relative to a normal value, at most
TINY = 2.0 ** -149        # the absolute spacing of binary32 subnormals
# stated accuracy of the approximate operators plus o32e's own rounding, as
# relative bounds: sin, cos, exp, log within 2 ulp (+ 1/2); the device
# library's tan, asin, acos, atan, tanh within 4 ulp (+ 1/2)
EPS_APPROX = {SIN: 4 * ULP, COS: 4 * ULP, EXP: 4 * ULP, LOG: 4 * ULP,
              TAN: 8 * ULP, ASIN: 8 * ULP, ACOS: 8 * ULP, ATAN: 8 * ULP, TANH: 8 * ULP}
EPS_SQRT = 2 * ULP        # faithful square root: 1.5 ulp from o32e's correctly rounded one
EPS_ROUNDED = ULP         # a correctly rounded operator on inexact operands


def _round32(v):
    with np.errstate(over="ignore", invalid="ignore"):
        return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def tape(tokens, consts, X, base: str = "o32e"):
    """Forward pass keeping every token's value vector and operand indices.

    base "o32e": every token's result rounded to binary32 (the oracle's
    fp32-emulating values); "o64": binary64 throughout.
    """
    X64 = np.asarray(X, dtype=np.float32).astype(np.float64)
    c64 = np.asarray(consts, dtype=np.float32).astype(np.float64)
    if base == "o64":
        return interp.run_tape(tokens, c64, X64)
    if base != "o32e":
        raise ValueError(base)
    M = X64.shape[0]
    values, children, pos = [], [], []
    for i, t in enumerate(tokens):
        op, arg = int(t) & 0xFF, int(t) >> 8
        if op == VAR:
            values.append(X64[:, arg].copy())
            children.append(())
        elif op == CONST:
            values.append(np.full(M, c64[arg]))
            children.append(())
        elif interp.ARITY[op] == 2:
            rb = pos.pop()
            ra = pos.pop()
            values.append(_round32(interp.apply_op(op, values[ra], values[rb], None)))
            children.append((ra, rb))
        else:
            rx = pos.pop()
            values.append(_round32(interp.apply_op(op, None, None, values[rx])))
            children.append((rx,))
        pos.append(i)
    return values, children


def token_eps(tokens, div_eps=None, eps_scale: float = 1.0):
    """(eps[t], always[t]): each token's relative error budget and whether it
    applies on every case (approximate operators, and DIV when div_eps is
    given) or only where an operand is inexact (correctly rounded ones).
    ``eps_scale`` multiplies every budget (small scales keep a perturbation
    test in the first-order regime)."""
    eps, always = [], []
    for tk in tokens:
        op = int(tk) & 0xFF
        if op in (VAR, CONST):
            e, a = 0.0, False
        elif op in EPS_APPROX:
            e, a = EPS_APPROX[op], True
        elif op == SQRT:
            e, a = EPS_SQRT, True
        elif op == DIV and div_eps is not None:
            e, a = div_eps, True
        else:
            e, a = EPS_ROUNDED, False
        eps.append(e * eps_scale)
        always.append(a)
    return eps, always


def case_bounds(tokens, consts, X, base: str = "o32e", div_eps=None, eps_scale: float = 1.0):
    """(values, children, d, rel) of one valid program: d[t] the per-case
    bound on |v'[t] - v[t]| (forward running bound, see the module header),
    rel[t] the per-case relative error budget of token t's own result (0
    where none applies)."""
    values, children = tape(tokens, consts, X, base)
    eps, always = token_eps(tokens, div_eps, eps_scale)
    L = len(tokens)
    M = values[0].shape[0]
    d = [None] * L
    rel = [None] * L
    with np.errstate(all="ignore"):
        for t in range(L):
            op = int(tokens[t]) & 0xFF
            kids = children[t]
            v = values[t]
            if not kids:
                d[t] = np.zeros(M)
                rel[t] = np.zeros(M)
                continue
            if len(kids) == 2:
                a, b = values[kids[0]], values[kids[1]]
                da, db = d[kids[0]], d[kids[1]]
                if op in (ADD, SUB):
                    p = da + db
                elif op == MUL:
                    p = np.abs(b) * da + np.abs(a) * db + da * db
                elif op == DIV:
                    ab = np.abs(b)
                    p = np.where(db < ab, (ab * da + np.abs(a) * db) / (ab * (ab - db)), np.inf)
                    p = np.where(b == 0.0, np.where(db == 0.0, 0.0, np.inf), p)
                else:
                    raise ValueError(op)
                exact = (da == 0.0) & (db == 0.0)
            else:
                x = values[kids[0]]
                dx = d[kids[0]]
                ax = np.abs(x)
                if op == SIN:
                    p = np.minimum(np.abs(np.cos(x)) * dx + 0.5 * dx * dx, 2.0)
                elif op == COS:
                    p = np.minimum(np.abs(np.sin(x)) * dx + 0.5 * dx * dx, 2.0)
                elif op == EXP:
                    e0 = np.exp(np.clip(x, -80.0, 80.0))
                    p = np.maximum(np.exp(np.clip(x + dx, -80.0, 80.0)) - e0,
                                   e0 - np.exp(np.clip(x - dx, -80.0, 80.0)))
                elif op == LOG:
                    p = np.where(dx < ax, np.log(ax / (ax - dx)), np.inf)
                    p = np.where(x == 0.0, np.where(dx == 0.0, 0.0, np.inf), p)
                elif op == SQRT:
                    p = np.maximum(np.sqrt(ax + dx) - np.sqrt(ax), np.sqrt(ax) - np.sqrt(np.maximum(ax - dx, 0.0)))
                elif op == SQUARE:
                    p = 2.0 * ax * dx + dx * dx
                elif op == RECIP:
                    p = np.where(dx < ax, dx / (ax * (ax - dx)), np.inf)
                elif op == TAN:
                    lo, hi = x - dx, x + dx
                    pole = np.floor(hi / np.pi - 0.5) != np.floor(lo / np.pi - 0.5)
                    p = np.where(pole, np.inf, dx * (1.0 + np.maximum(np.tan(lo) ** 2, np.tan(hi) ** 2)))
                elif op in (ASIN, ACOS):
                    m = ax + dx
                    p = np.where(m < 1.0, dx / np.sqrt(1.0 - m * m), np.inf)
                elif op == ATAN:
                    p = np.minimum(dx, np.pi)
                elif op == TANH:
                    p = np.minimum(dx, 2.0)
                else:
                    raise ValueError(op)
                exact = dx == 0.0
            p = np.where(np.isnan(p), np.inf, p)
            r = np.full(M, eps[t]) if always[t] else np.where(exact, 0.0, eps[t])
            rel[t] = r
            d[t] = p + np.where(r > 0.0, r * (np.abs(v) + p) + TINY, 0.0)
    return values, children, d, rel


def mse_bound(y_hat, y, b) -> float:
    """Largest change of the MSE when every output moves by at most b[i]."""
    yh = np.asarray(y_hat, dtype=np.float64)
    y64 = np.asarray(y, dtype=np.float32).astype(np.float64)
    if not np.all(np.isfinite(b)):
        return math.inf
    with np.errstate(all="ignore"):
        B = float(np.sum(2.0 * np.abs(yh - y64) * b + b * b)) / yh.shape[0]
    return B if math.isfinite(B) else math.inf


def corr_bound(y_hat, y, b) -> float:
    """Largest change of 1 - r^2 (non-constant outputs) when every output
    moves by at most b[i] (see the module header)."""
    yh = np.asarray(y_hat, dtype=np.float64)
    y64 = np.asarray(y, dtype=np.float32).astype(np.float64)
    if not np.all(np.isfinite(b)):
        return math.inf
    M = yh.shape[0]
    sxx, syy, sxy = ofit.pearson_sums(yh, y64)
    s = math.sqrt(sxx)
    r = sxy / math.sqrt(sxx * syy)
    u = yh - math.fsum(yh.tolist()) / M
    w = y64 - math.fsum(y64.tolist()) / M
    B1 = float(np.sum(np.abs(w / math.sqrt(sxx * syy) - r * u / sxx) * b))
    g = float(np.sqrt(np.sum(b * b)))
    if not g < s:
        return math.inf
    Br = (s * B1 + abs(r) * g * g / (2.0 * (s - g))) / (s - g)
    B = min(Br * (2.0 * abs(r) + Br), 1.0)
    return B if math.isfinite(B) else math.inf


def fitness_bound(tokens, consts, X, y, kind: int, base: str = "o32e", div_eps=None,
                  eps_scale: float = 1.0) -> float:
    """B of one valid program (see the module header): +inf when no bound
    exists, NaN when the base fitness is not finite."""
    values, children, d, _ = case_bounds(tokens, consts, X, base, div_eps, eps_scale)
    yh = values[-1]
    F = ofit.fitness(kind, yh, y)
    if not math.isfinite(F):
        return math.nan
    if kind == ofit.MSE:
        return mse_bound(yh, y, d[-1])
    if np.all(yh == yh[0]):
        # a constant output: F = 1 by convention, any variation gives some r
        varying = any(np.any(d[t] > 0.0) and not np.all(values[t] == values[t][0]) for t in range(len(tokens)))
        return math.inf if varying else 0.0
    return corr_bound(yh, y, d[-1])


def seed(kind: int, y_hat, y):
    """(F, dF/dyhat) in binary64 at the given outputs."""
    yh = np.asarray(y_hat, dtype=np.float64)
    y64 = np.asarray(y, dtype=np.float32).astype(np.float64)
    M = yh.shape[0]
    F = ofit.fitness(kind, yh, y64)
    if not math.isfinite(F):
        return F, None
    if kind == ofit.MSE:
        return F, 2.0 * (yh - y64) / M
    sxx, syy, sxy = ofit.pearson_sums(yh, y64)
    if sxx == 0.0:
        return F, np.zeros(M)
    r = sxy / math.sqrt(sxx * syy)
    u = yh - math.fsum(yh.tolist()) / M
    w = y64 - math.fsum(y64.tolist()) / M
    return F, -2.0 * r * (w / math.sqrt(sxx * syy) - r * u / sxx)


def adjoints(tokens, values, children, seed_vec):
    """Per-token adjoint vectors A[t] = dF/dv[t] (reverse sweep, binary64,
    the partial derivatives of the operator conventions; 0 at a protected
    operator's branch point): the first-order effect of an error on token
    t's result, whose signs give the worst-case errors."""
    L = len(tokens)
    adj = [None] * L
    adj[L - 1] = seed_vec
    with np.errstate(all="ignore"):
        for t in range(L - 1, -1, -1):
            op = int(tokens[t]) & 0xFF
            a_t = adj[t]
            kids = children[t]
            if not kids:
                continue
            if len(kids) == 2:
                ia, ib = kids
                a, b = values[ia], values[ib]
                if op == ADD:
                    da, db = a_t, a_t
                elif op == SUB:
                    da, db = a_t, -a_t
                elif op == MUL:
                    da, db = a_t * b, a_t * a
                elif op == DIV:
                    on = b == 0.0
                    bs = np.where(on, 1.0, b)
                    da = np.where(on, 0.0, a_t / bs)
                    db = np.where(on, 0.0, -a_t * a / (bs * bs))
                else:
                    raise ValueError(op)
                adj[ia], adj[ib] = da, db
            else:
                (ix,) = kids
                x = values[ix]
                if op == SIN:
                    dfx = np.cos(x)
                elif op == COS:
                    dfx = -np.sin(x)
                elif op == EXP:
                    inside = ~((x > 80.0) | (x < -80.0))
                    dfx = np.where(inside, np.exp(np.where(inside, x, 0.0)), 0.0)
                elif op in (LOG, SQRT):
                    on = x == 0.0
                    xs = np.where(on, 1.0, x)
                    dfx = 1.0 / xs if op == LOG else np.sign(xs) / (2.0 * np.sqrt(np.abs(xs)))
                    dfx = np.where(on, 0.0, dfx)
                elif op == SQUARE:
                    dfx = 2.0 * x
                elif op == RECIP:
                    dfx = -1.0 / (x * x)
                elif op == TAN:
                    tx = np.tan(x)
                    dfx = 1.0 + tx * tx
                elif op in (ASIN, ACOS):
                    dfx = 1.0 / np.sqrt(1.0 - x * x)
                    dfx = dfx if op == ASIN else -dfx
                elif op == ATAN:
                    dfx = 1.0 / (1.0 + x * x)
                elif op == TANH:
                    e = np.exp(-2.0 * np.abs(x))
                    dfx = 4.0 * e / ((1.0 + e) * (1.0 + e))
                else:
                    raise ValueError(op)
                adj[ix] = np.where(a_t == 0.0, 0.0, a_t * dfx)
    return adj
