"""First-order bound on the fitness change of a binary32 evaluation -- test infrastructure.

Why it exists.  The parity claim of the library is a binary32 evaluation per
case (paper, section 2.1.2: every genome is run on every fitness case) whose
+ - * / are correctly rounded and whose other operators are accurate to a
few ulps.  Such an evaluation reproduces the fp32-emulating oracle (mode
"o32e" of ``oracle.interp``) token by token except that each token's result
may carry a small relative error of its own.  How far that moves a program's
fitness depends on the program: sin of a large argument or exp of a large
argument amplifies it enormously.  This module computes, for one program, a
bound B on that movement, so that every program can be value-checked
against the oracle, the ill-conditioned ones included, with an envelope
that follows from the stated operator accuracies rather than from a
tolerance chosen by hand.

Model.  Token t on case i has the value v[t,i] along a base trajectory (the
o32e values by default).  The evaluation under test computes
v[t,i] (1 + d[t,i]) instead, |d[t,i]| <= eps[t], and everything downstream
takes the perturbed value.  To first order the fitness then moves by

    dF = sum over t, i of  A[t,i] v[t,i] d[t,i],

where A[t,i] = dF / dv[t,i] is token t's adjoint on case i: the derivative
of the fitness with respect to that token's output through everything that
consumes it (reverse mode over the postfix tape; Linnainmaa, BIT 16 (1976),
introduced reverse accumulation exactly for this estimate of accumulated
rounding error).  Hence

    |dF| <= B = sum over t, i of  |A[t,i]| (|v[t,i]| eps[t] + tiny[t]),

with tiny[t] = 2^-149 (the absolute error of a binary32 subnormal result)
where eps[t] > 0.

eps per token (``token_eps``), for a binary32 evaluation against o32e:
  * VAR, CONST: 0 (the same binary32 inputs).
  * SIN COS EXP LOG and the five further library functions: their stated
    accuracy plus o32e's own half ulp, as a relative bound (``EPS_APPROX``).
  * SQRT: faithful (within 1 ulp of the exact value, o32e within 1/2):
    1.5 ulp < 2^-22.
  * ADD SUB MUL DIV SQUARE RECIP (correctly rounded): 0 when every input is
    bit-identical to o32e, i.e. when no token below it carries an error
    ("untainted"); otherwise the two roundings of slightly different exact
    values can differ by up to 1 ulp: 2^-23.  ``div_eps`` overrides DIV for
    an implementation whose division is not correctly rounded.
A constant output under 1 - r^2 is a branch point too (F = 1 by
convention, any variation gives some r): B is 0 when every token carrying
error has one value on all cases, +inf otherwise.
The protected operators have branch points (DIV with b == 0, LOG with
x == 0, SQRT at 0 with its unbounded derivative).  A tainted input lying
exactly on such a point may move off it, and the fitness jumps: no
first-order bound exists, and B is +inf ("vacuous").  An untainted input at
such a point stays there; its branch's derivative is then irrelevant and
taken as 0.  Where a partial derivative or a product is not finite, B is
+inf as well.

Seeds dF/dyhat_i (binary64, at the base trajectory's yhat):
  MSE   2 (yhat_i - y_i) / M
  CORR  -2 r (w_i / sqrt(Sxx Syy) - r u_i / Sxx) with the centred sums of
        Eq. 1 (u = yhat - mean yhat, w = y - mean y); 0 when Sxx == 0 (F is
        then 1 by convention).
Partial derivatives: those of the operator conventions in ``oracle.interp``,
evaluated in binary64 at the base values:
  ADD (1, 1)  SUB (1, -1)  MUL (b, a)  DIV (1/b, -a/b^2)
  SIN cos x  COS -sin x  EXP e^x inside [-80, 80], 0 outside
  LOG 1/x  SQRT sign(x) / (2 sqrt|x|)  SQUARE 2x  RECIP -1/x^2
  TAN 1 + tan^2 x  ASIN 1/sqrt(1 - x^2)  ACOS -1/sqrt(1 - x^2)
  ATAN 1/(1 + x^2)  TANH 4e/(1 + e)^2 with e = exp(-2|x|)
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
EPS_ROUNDED = ULP         # a correctly rounded operator on tainted inputs


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


def token_eps(tokens, children, div_eps=None, eps_scale: float = 1.0):
    """(eps[t], tainted[t]) for every token (see the module header);
    ``eps_scale`` multiplies every eps (small scales keep a perturbation
    test in the first-order regime)."""
    eps = [0.0] * len(tokens)
    tainted = [False] * len(tokens)
    for t, tk in enumerate(tokens):
        op = int(tk) & 0xFF
        below = any(tainted[c] for c in children[t])
        if op in (VAR, CONST):
            e = 0.0
        elif op in EPS_APPROX:
            e = EPS_APPROX[op]
        elif op == SQRT:
            e = EPS_SQRT
        elif op == DIV and div_eps is not None:
            e = max(div_eps, EPS_ROUNDED if below else 0.0)
        else:
            e = EPS_ROUNDED if below else 0.0
        eps[t] = e * eps_scale
        tainted[t] = below or e > 0.0
    return eps, tainted


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


def adjoints(tokens, values, children, seed_vec, tainted):
    """Per-token adjoint vectors A[t] = dF/dv[t] (reverse sweep, binary64);
    None when a tainted input sits on a protected operator's branch point."""
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
            if a_t is None:
                a_t = np.zeros_like(seed_vec)
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
                    if np.any(on & (a_t != 0.0)) and tainted[ib]:
                        return None
                    bs = np.where(on, 1.0, b)
                    da = np.where(on, 0.0, a_t / bs)
                    db = np.where(on, 0.0, -a_t * a / (bs * bs))
                else:
                    raise ValueError(op)
                adj[ia] = da if adj[ia] is None else adj[ia] + da
                adj[ib] = db if adj[ib] is None else adj[ib] + db
            else:
                (ix,) = kids
                x = values[ix]
                if op == SIN:
                    d = np.cos(x)
                elif op == COS:
                    d = -np.sin(x)
                elif op == EXP:
                    inside = ~((x > 80.0) | (x < -80.0))
                    d = np.where(inside, np.exp(np.where(inside, x, 0.0)), 0.0)
                elif op in (LOG, SQRT):
                    on = x == 0.0
                    if np.any(on & (a_t != 0.0)) and tainted[ix]:
                        return None
                    xs = np.where(on, 1.0, x)
                    d = 1.0 / xs if op == LOG else np.sign(xs) / (2.0 * np.sqrt(np.abs(xs)))
                    d = np.where(on, 0.0, d)
                elif op == SQUARE:
                    d = 2.0 * x
                elif op == RECIP:
                    d = -1.0 / (x * x)
                elif op == TAN:
                    tx = np.tan(x)
                    d = 1.0 + tx * tx
                elif op in (ASIN, ACOS):
                    d = 1.0 / np.sqrt(1.0 - x * x)
                    d = d if op == ASIN else -d
                elif op == ATAN:
                    d = 1.0 / (1.0 + x * x)
                elif op == TANH:
                    e = np.exp(-2.0 * np.abs(x))
                    d = 4.0 * e / ((1.0 + e) * (1.0 + e))
                else:
                    raise ValueError(op)
                dx = np.where(a_t == 0.0, 0.0, a_t * d)
                adj[ix] = dx if adj[ix] is None else adj[ix] + dx
    return adj


def fitness_bound(tokens, consts, X, y, kind: int, base: str = "o32e", div_eps=None,
                  eps_scale: float = 1.0) -> float:
    """B of one valid program (see the module header): +inf when no
    first-order bound exists, NaN when the base fitness is not finite."""
    values, children = tape(tokens, consts, X, base)
    F, sv = seed(kind, values[-1], y)
    if sv is None:
        return math.nan
    eps, tainted = token_eps(tokens, children, div_eps, eps_scale)
    if kind == ofit.CORR and np.all(values[-1] == values[-1][0]):
        # a constant output: F = 1 by convention, and any case-to-case
        # variation, however small, gives some r.  The output stays constant
        # when every token that carries error has one value on all cases
        # (the same operation on the same operands); otherwise F is not
        # determined at all.
        varying = any(tainted[t] and not np.all(values[t] == values[t][0]) for t in range(len(tokens)))
        return math.inf if varying else 0.0
    adj = adjoints(tokens, values, children, sv, tainted)
    if adj is None:
        return math.inf
    terms = []
    with np.errstate(all="ignore"):
        for t in range(len(tokens)):
            if eps[t] == 0.0 or adj[t] is None:
                continue
            a = np.abs(adj[t])
            c = np.where(a == 0.0, 0.0, a * (np.abs(values[t]) * eps[t] + TINY))
            if not np.all(np.isfinite(c)):
                return math.inf
            terms.append(float(np.sum(c)))  # non-negative terms: pairwise sum suffices for a bound
    B = math.fsum(terms)
    return B if math.isfinite(B) else math.inf
