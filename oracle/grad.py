"""Gradient of the fitness with respect to program constants -- test infrastructure.

The paper evolves structure and constants together and has no gradient step;
the library adds a reverse-mode adjoint over the postfix tape so a program's
ephemeral constants can be tuned by gradient descent.  This module is the
float64 reference for it.

Seeds dF/dy_hat_i:
  MSE   F = (1/M) sum_i (y_hat_i - y_i)^2:  2 (y_hat_i - y_i) / M.
  CORR  F = 1 - r^2 with r Pearson's coefficient (Eq. 1) of y_hat and y,
        from the centred sums Sxx, Syy, Sxy (u_i = y_hat_i - mean y_hat,
        w_i = y_i - mean y):
            dr/dy_hat_i = w_i / sqrt(Sxx Syy) - r u_i / Sxx,
            dF/dy_hat_i = -2 r dr/dy_hat_i.
        Readings: the derivative is that of 1 - r^2 also where F is clamped
        to [0, 1] (rounding only); Sxx == 0 (F = 1 by convention): 0; a NaN
        fitness gives NaN seeds.
Adjoints flow from each token to its operands (reverse token order) with
these partial derivatives, matching the operator conventions of
``oracle.interp`` (derivative taken as 0 where a protected branch replaces
the operator by a constant):
  ADD (1, 1)   SUB (1, -1)   MUL (b, a)
  DIV (1/b, -a/b^2) if b != 0, else (0, 0)
  SIN cos x    COS -sin x
  EXP exp x inside [-80, 80], else 0
  LOG 1/x if x != 0, else 0
  SQRT sign(x) / (2 sqrt|x|) if x != 0, else 0
  SQUARE 2x      RECIP -1/x^2      TAN 1 + tan^2 x
  ASIN 1/sqrt(1 - x^2)   ACOS -1/sqrt(1 - x^2)   (NaN outside [-1, 1])
  ATAN 1/(1 + x^2)       TANH sech^2 x = 4e / (1 + e)^2, e = exp(-2|x|)
                         (1 - tanh^2 x cancels where tanh saturates)
A constant slot's gradient is the sum over cases of the adjoints of every
CONST token that reads it.

Modes (conditioning only; the reference gradient is "o64"):
  "o32e"  every forward value, every partial derivative and every adjoint
          product rounded to binary32 (the per-case arithmetic of an fp32
          adjoint), sums over cases still exact;
  "o32p"  as o32e, with the results of the approximate operators
          (oracle.interp.APPROXIMATE) and the derivative values computed from
          transcendental functions perturbed by a few ulps (seeded), as in
          oracle.interp.
In the fp32 modes the further operators' derivatives are formed from the
rounded values the way an fp32 adjoint forms them: SQUARE 2x, RECIP -(y y),
TAN 1 + y y, ASIN and ACOS +-1/sqrt((1 - x)(1 + x)) (approximate),
ATAN 1/(1 + x x), TANH 4e / ((1 + e)(1 + e)) with e = exp(max(-2|x|, -80))
(approximate), with y the operator's value.
A gradient component is stable under these modes when an fp32 adjoint can
reproduce it; where per-case contributions cancel it is not.
"""
from __future__ import annotations

import math

import numpy as np

from . import fitness as ofit
from . import interp

ADD, SUB, MUL, DIV, SIN, COS, EXP, LOG, SQRT, VAR, CONST = range(11)
SQUARE, RECIP, TAN, ASIN, ACOS, ATAN, TANH = range(11, 18)


def _fsum(v) -> float:
    """Exactly rounded sum; plain IEEE sum when a term is not finite."""
    arr = np.asarray(v, dtype=np.float64)
    if np.all(np.isfinite(arr)):
        return math.fsum(arr.tolist())
    with np.errstate(all="ignore"):
        return float(np.sum(arr))


def _mse64(y_hat, y64):
    d = y_hat - y64
    return math.fsum((d * d).tolist()) / y_hat.shape[0]


def mse_and_grad(tokens, consts, X, y, mode: str = "o64", seed: int = 0):
    """(F, dF/dconsts float64[len(consts)]); binary64 throughout for "o64"."""
    X64 = np.asarray(X, dtype=np.float32).astype(np.float64)
    y64 = np.asarray(y, dtype=np.float32).astype(np.float64)
    c64 = np.asarray(consts, dtype=np.float32).astype(np.float64)
    return mse_and_grad64(tokens, c64, X64, y64, mode, seed)


def _rounder(mode, seed, M):
    if mode == "o64":
        return (lambda v: v), (lambda v: v)
    rng = np.random.default_rng(seed)

    def r32(v):
        with np.errstate(over="ignore", invalid="ignore"):
            return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)

    def r32t(v):  # a transcendental result
        if mode == "o32p":
            with np.errstate(all="ignore"):
                v = v * (1.0 + rng.uniform(-2.0 ** -22, 2.0 ** -22, size=M))
        return r32(v)

    return r32, r32t


def corr_and_grad(tokens, consts, X, y, mode: str = "o64", seed: int = 0):
    """(1 - r^2, dF/dconsts float64[len(consts)]); binary64 throughout for "o64"."""
    X64 = np.asarray(X, dtype=np.float32).astype(np.float64)
    y64 = np.asarray(y, dtype=np.float32).astype(np.float64)
    c64 = np.asarray(consts, dtype=np.float32).astype(np.float64)
    return fitness_and_grad64(CORR_KIND, tokens, c64, X64, y64, mode, seed)


MSE_KIND, CORR_KIND = 0, 1


def _corr_seed(y_hat, y64):
    """(F, dF/dy_hat) of F = 1 - r^2, binary64, with the readings above."""
    F = ofit.corr_fitness(y_hat, y64)
    M = y_hat.shape[0]
    if not math.isfinite(F):
        return F, np.full(M, math.nan)
    sxx, syy, sxy = ofit.pearson_sums(y_hat, y64)
    if sxx == 0.0:
        return F, np.zeros(M)
    r = sxy / math.sqrt(sxx * syy)
    u = y_hat - math.fsum(y_hat.tolist()) / M
    w = y64 - math.fsum(y64.tolist()) / M
    return F, -2.0 * r * (w / math.sqrt(sxx * syy) - r * u / sxx)


def mse_and_grad64(tokens, c64, X64, y64, mode: str = "o64", seed: int = 0):
    return fitness_and_grad64(MSE_KIND, tokens, c64, X64, y64, mode, seed)


def fitness_and_grad64(kind, tokens, c64, X64, y64, mode: str = "o64", seed: int = 0):
    """(F, gradient): the fitness kind's seed, then the reverse sweep."""
    M = X64.shape[0]
    L = len(tokens)
    R, RT = _rounder(mode, seed, M)
    if mode == "o64":
        values, children = interp.run_tape(tokens, c64, X64)
    else:
        values, children = _tape_rounded(tokens, c64, X64, R, RT)
    y_hat = values[-1]
    adj = [None] * L
    if kind == MSE_KIND:
        F = _mse64(y_hat, y64)
        adj[L - 1] = R(R(y_hat - y64) * R(2.0 / M)) if mode != "o64" else 2.0 * (y_hat - y64) / M
    else:
        with np.errstate(all="ignore"):
            F, sd = _corr_seed(y_hat, y64)
        adj[L - 1] = R(sd)
    g = [[] for _ in range(len(c64))]
    with np.errstate(all="ignore"):
        for t in range(L - 1, -1, -1):
            op, arg = int(tokens[t]) & 0xFF, int(tokens[t]) >> 8
            a_t = adj[t]
            if op == VAR:
                continue
            if op == CONST:
                g[arg].append(_fsum(a_t))
                continue
            kids = children[t]
            if len(kids) == 2:
                ia, ib = kids
                a, b = values[ia], values[ib]
                if op == ADD:
                    da, db = a_t, a_t
                elif op == SUB:
                    da, db = a_t, -a_t
                elif op == MUL:
                    da, db = R(a_t * b), R(a_t * a)
                elif op == DIV:
                    nz = b != 0.0
                    bs = np.where(nz, b, 1.0)
                    if mode == "o64":
                        da = np.where(nz, a_t / bs, 0.0)
                        db = np.where(nz, -a_t * a / (bs * bs), 0.0)
                    else:
                        r = R(1.0 / bs)
                        da = np.where(nz, R(a_t * r), 0.0)
                        db = np.where(nz, R(a_t * R(R(-a * r) * r)), 0.0)
                else:
                    raise ValueError(op)
                adj[ia], adj[ib] = da, db
            else:
                (ix,) = kids
                x = values[ix]
                if mode == "o64":
                    if op == SIN:
                        dx = a_t * np.cos(x)
                    elif op == COS:
                        dx = -a_t * np.sin(x)
                    elif op == EXP:
                        inside = ~((x > 80.0) | (x < -80.0))
                        dx = np.where(inside, a_t * np.exp(np.where(inside, x, 0.0)), 0.0)
                    elif op == LOG:
                        nz = x != 0.0
                        dx = np.where(nz, a_t / np.where(nz, x, 1.0), 0.0)
                    elif op == SQRT:
                        nz = x != 0.0
                        dx = np.where(nz, a_t * np.sign(x) / (2.0 * np.sqrt(np.abs(np.where(nz, x, 1.0)))), 0.0)
                    elif op == SQUARE:
                        dx = a_t * (2.0 * x)
                    elif op == RECIP:
                        dx = -a_t / (x * x)
                    elif op == TAN:
                        t_x = np.tan(x)
                        dx = a_t * (1.0 + t_x * t_x)
                    elif op in (ASIN, ACOS):
                        d = 1.0 / np.sqrt(1.0 - x * x)
                        dx = a_t * (d if op == ASIN else -d)
                    elif op == ATAN:
                        dx = a_t / (1.0 + x * x)
                    elif op == TANH:
                        e = np.exp(-2.0 * np.abs(x))
                        dx = a_t * (4.0 * e / ((1.0 + e) * (1.0 + e)))
                    else:
                        raise ValueError(op)
                else:
                    yv = values[t]
                    if op == SIN:
                        d = RT(np.cos(x))
                    elif op == COS:
                        d = -RT(np.sin(x))
                    elif op == EXP:
                        d = np.where((x > 80.0) | (x < -80.0), 0.0, yv)
                    elif op == LOG:
                        d = np.where(x != 0.0, R(1.0 / np.where(x != 0.0, x, 1.0)), 0.0)
                    elif op == SQRT:
                        d = np.where(x != 0.0, R(np.copysign(0.5, x) / np.where(x != 0.0, yv, 1.0)), 0.0)
                    elif op == SQUARE:
                        d = R(2.0 * x)
                    elif op == RECIP:
                        d = R(-(yv * yv))
                    elif op == TAN:
                        d = R(1.0 + R(yv * yv))
                    elif op in (ASIN, ACOS):
                        d = RT(1.0 / np.sqrt(R(R(1.0 - x) * R(1.0 + x))))
                        d = d if op == ASIN else -d
                    elif op == ATAN:
                        d = R(1.0 / R(1.0 + R(x * x)))
                    elif op == TANH:
                        e = RT(np.exp(np.maximum(R(-2.0 * np.abs(x)), -80.0)))
                        ep = R(1.0 + e)
                        d = R(R(4.0 * e) / R(ep * ep))
                    else:
                        raise ValueError(op)
                    dx = R(a_t * d)
                adj[ix] = dx
    grad = np.array([_fsum(v) for v in g], dtype=np.float64)
    return F, grad


def _tape_rounded(tokens, c64, X64, R, RT):
    """run_tape with every result rounded to binary32 (RT for sin/cos/exp/log)."""
    M = X64.shape[0]
    X32 = R(X64)
    values = []
    children = []
    pos_stack = []
    for i, t in enumerate(tokens):
        op, arg = int(t) & 0xFF, int(t) >> 8
        if op == VAR:
            values.append(X32[:, arg].copy())
            children.append(())
        elif op == CONST:
            values.append(np.full(M, float(R(np.array([c64[arg]]))[0])))
            children.append(())
        elif interp.ARITY[op] == 2:
            rb = pos_stack.pop()
            ra = pos_stack.pop()
            values.append(R(interp.apply_op(op, values[ra], values[rb], None)))
            children.append((ra, rb))
        else:
            rx = pos_stack.pop()
            v = interp.apply_op(op, None, None, values[rx])
            values.append(RT(v) if op in interp.APPROXIMATE else R(v))
            children.append((rx,))
        pos_stack.append(i)
    return values, children


def branch_masks(tokens, c64, X64):
    """Boolean masks of every protected-branch decision (for FD admissibility)."""
    values, children = interp.run_tape(tokens, c64, X64)
    masks = []
    for t, tk in enumerate(tokens):
        op = int(tk) & 0xFF
        if op == DIV:
            masks.append(values[children[t][1]] == 0.0)
        elif op == EXP:
            x = values[children[t][0]]
            masks.append(x > 80.0)
            masks.append(x < -80.0)
        elif op == LOG or op == SQRT:
            masks.append(values[children[t][0]] == 0.0)
    return masks


def central_fd(tokens, consts, X, y, rel_step: float = 1e-5, kind: int = MSE_KIND):
    """Central finite differences of the binary64 fitness, and which slots are admissible.

    Step h_j = rel_step * max(1, |c_j|).  A slot is inadmissible when the +-h
    perturbation flips any protected-branch decision in any case.
    """
    X64 = np.asarray(X, dtype=np.float32).astype(np.float64)
    y64 = np.asarray(y, dtype=np.float32).astype(np.float64)
    c64 = np.asarray(consts, dtype=np.float32).astype(np.float64)
    base = branch_masks(tokens, c64, X64)
    fd = np.zeros(len(c64))
    ok = np.ones(len(c64), dtype=bool)
    for j in range(len(c64)):
        h = rel_step * max(1.0, abs(c64[j]))
        cp = c64.copy()
        cm = c64.copy()
        cp[j] += h
        cm[j] -= h
        for cc in (cp, cm):
            for m0, m1 in zip(base, branch_masks(tokens, cc, X64)):
                if np.any(m0 != m1):
                    ok[j] = False
        fit = _mse64 if kind == MSE_KIND else ofit.corr_fitness
        fp = fit(interp.run_tape(tokens, cp, X64)[0][-1], y64)
        fm = fit(interp.run_tape(tokens, cm, X64)[0][-1], y64)
        fd[j] = (fp - fm) / (cp[j] - cm[j])
    return fd, ok
