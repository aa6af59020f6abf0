"""Postfix stack interpreter -- test infrastructure (see oracle/__init__.py).

The genome is a reverse-Polish program (paper, section 2.1.4): terminals push
a value, operators pop their operands and push the result.  All lanes of the
paper's GPU kernel run one program over many fitness cases (section 2.1.2);
here the same thing is written as one numpy vector per stack entry, one
element per fitness case.

Token format: uint16 ``opcode | (arg << 8)``.
Opcodes: 0 ADD 1 SUB 2 MUL 3 DIV 4 SIN 5 COS 6 EXP 7 LOG 8 SQRT
9 VAR (arg = input variable) 10 CONST (arg = constant slot), and the rest
of the paper's operator table (its parameter table, section 2.1.7):
11 SQUARE 12 RECIP 13 TAN 14 ASIN 15 ACOS 16 ATAN 17 TANH (unary).
For a binary operator the top of the stack is the right operand b and the
entry below it the left operand a; the result is ``a op b``.

Operator conventions (the paper keeps invalid values instead of protecting
operators; the library fixes these protected forms):
  DIV   b == 0 ? 1 : a / b          (exact zero test; -0 == 0)
  SIN   sin(x), COS cos(x)          (+-Inf -> NaN)
  EXP   exp(min(max(x, -80), 80)) written with comparisons, so NaN -> NaN
  LOG   x == 0 ? 0 : log|x|
  SQRT  sqrt|x|
The seven further operators keep the paper's unprotected semantics (invalid
values flow on and are scored as such, section 2.1.5):
  SQUARE x * x        RECIP 1 / x (+-Inf at +-0)
  TAN   tan x (+-Inf -> NaN)
  ASIN, ACOS  NaN outside [-1, 1]
  ATAN  atan x        TANH tanh x

Modes
  "o64"  every operation in IEEE binary64 on the fp32 inputs widened exactly
  "o32e" identical, but each token's result is rounded to binary32 (round to
         nearest even, overflow to Inf).  For + - * / sqrt this equals IEEE
         fp32 arithmetic exactly (binary64 has more than 2*24+2 bits, so the
         double rounding is innocuous); for sin, cos, exp, log it is the
         binary64 libm value rounded once.
  "o32p" o32e with the binary64 result of every sin, cos, exp, log,
         sqrt, tan, asin, acos, atan and tanh token first scaled by (1 + e), e uniform in [-2^-22, 2^-22] (a
         few binary32 ulps), drawn from a seeded generator: a model of a
         binary32 implementation whose + - * / are correctly rounded and whose
         other operators are accurate to a few ulps.  Used only to
         decide whether a program's fitness is stable under such differences
         (conditioning), never as a reference value.
"""
from __future__ import annotations

import numpy as np

ADD, SUB, MUL, DIV, SIN, COS, EXP, LOG, SQRT, VAR, CONST = range(11)
SQUARE, RECIP, TAN, ASIN, ACOS, ATAN, TANH = range(11, 18)
N_OPCODES = 18
EXTENDED = (SQUARE, RECIP, TAN, ASIN, ACOS, ATAN, TANH)
ARITY = {ADD: 2, SUB: 2, MUL: 2, DIV: 2, SIN: 1, COS: 1, EXP: 1, LOG: 1, SQRT: 1, VAR: 0, CONST: 0}
ARITY.update({op: 1 for op in EXTENDED})
# results of these operators come from approximate (few-ulp) device functions
APPROXIMATE = (SIN, COS, EXP, LOG, SQRT, TAN, ASIN, ACOS, ATAN, TANH)

# per-program status codes
ST_OK = 0
ST_EMPTY = 1
ST_BAD_OPCODE = 2
ST_UNDERFLOW = 3
ST_BAD_FINAL_DEPTH = 4
ST_BAD_VAR = 5
ST_BAD_CONST = 6
ST_TOO_LONG = 7

MAX_LEN = 4096
EXP_CLAMP = 80.0


def validate(tokens, const_count: int, D: int):
    """Check the stack discipline and operand ranges of one program.

    Returns (status, max_depth).  Tokens are scanned in order; the first
    faulty token decides the status, checking in this order: opcode range,
    variable index < D, constant slot < const_count, stack underflow.  A
    program with no faulty token must end with exactly one value on the stack.
    """
    L = len(tokens)
    if L == 0:
        return ST_EMPTY, 0
    if L > MAX_LEN:
        return ST_TOO_LONG, 0
    depth = 0
    max_depth = 0
    for t in tokens:
        op, arg = int(t) & 0xFF, int(t) >> 8
        if op >= N_OPCODES:
            return ST_BAD_OPCODE, max_depth
        if op == VAR and arg >= D:
            return ST_BAD_VAR, max_depth
        if op == CONST and arg >= const_count:
            return ST_BAD_CONST, max_depth
        a = ARITY[op]
        if depth < a:
            return ST_UNDERFLOW, max_depth
        depth += 1 - a
        max_depth = max(max_depth, depth)
    if depth != 1:
        return ST_BAD_FINAL_DEPTH, max_depth
    return ST_OK, max_depth


def _round32(v: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        return v.astype(np.float32).astype(np.float64)


def apply_op(op: int, a, b, x):
    """One operator on float64 vectors.  Binary: a (left), b (right); unary: x."""
    with np.errstate(all="ignore"):
        if op == ADD:
            return a + b
        if op == SUB:
            return a - b
        if op == MUL:
            return a * b
        if op == DIV:
            return np.where(b == 0.0, 1.0, a / np.where(b == 0.0, 1.0, b))
        if op == SIN:
            return np.sin(x)
        if op == COS:
            return np.cos(x)
        if op == EXP:
            c = np.where(x > EXP_CLAMP, EXP_CLAMP, np.where(x < -EXP_CLAMP, -EXP_CLAMP, x))
            return np.exp(c)
        if op == LOG:
            return np.where(x == 0.0, 0.0, np.log(np.where(x == 0.0, 1.0, np.abs(x))))
        if op == SQRT:
            return np.sqrt(np.abs(x))
        if op == SQUARE:
            return x * x
        if op == RECIP:
            return 1.0 / x
        if op == TAN:
            return np.tan(x)
        if op == ASIN:
            return np.arcsin(x)
        if op == ACOS:
            return np.arccos(x)
        if op == ATAN:
            return np.arctan(x)
        if op == TANH:
            return np.tanh(x)
    raise ValueError(f"not an operator: {op}")


def run(tokens, consts, X, mode: str = "o64", seed: int = 0) -> np.ndarray:
    """Evaluate one valid program on every row of X; returns y_hat float64 [M].

    ``consts`` and ``X`` are the fp32 arrays the GPU receives; they are
    widened to binary64 exactly.  ``seed`` drives the "o32p" perturbations.
    """
    if mode not in ("o64", "o32e", "o32p"):
        raise ValueError(mode)
    rng = np.random.default_rng(seed) if mode == "o32p" else None
    X64 = np.asarray(X, dtype=np.float32).astype(np.float64)
    c64 = np.asarray(consts, dtype=np.float32).astype(np.float64)
    M = X64.shape[0]
    stack = []
    for t in tokens:
        op, arg = int(t) & 0xFF, int(t) >> 8
        if op == VAR:
            stack.append(X64[:, arg].copy())
            continue
        if op == CONST:
            stack.append(np.full(M, c64[arg]))
            continue
        if ARITY[op] == 2:
            b = stack.pop()
            a = stack.pop()
            v = apply_op(op, a, b, None)
        else:
            v = apply_op(op, None, None, stack.pop())
        if mode == "o32p" and op in APPROXIMATE:
            with np.errstate(all="ignore"):
                v = v * (1.0 + rng.uniform(-2.0 ** -22, 2.0 ** -22, size=M))
        if mode != "o64":
            v = _round32(v)
        stack.append(v)
    (y_hat,) = stack
    return y_hat


def run_tape(tokens, consts64, X64: np.ndarray):
    """Binary64 forward pass keeping every token's value (the tape).

    ``consts64`` may hold arbitrary binary64 values (finite differences
    perturb them).  Returns (values, children): values[t] is token t's output
    vector, children[t] the token indices of its operands (left, right).
    """
    M = X64.shape[0]
    values = []
    children = []
    pos_stack = []
    for i, t in enumerate(tokens):
        op, arg = int(t) & 0xFF, int(t) >> 8
        if op == VAR:
            values.append(X64[:, arg].copy())
            children.append(())
        elif op == CONST:
            values.append(np.full(M, float(consts64[arg])))
            children.append(())
        elif ARITY[op] == 2:
            rb = pos_stack.pop()
            ra = pos_stack.pop()
            values.append(apply_op(op, values[ra], values[rb], None))
            children.append((ra, rb))
        else:
            rx = pos_stack.pop()
            values.append(apply_op(op, None, None, values[rx]))
            children.append((rx,))
        pos_stack.append(i)
    return values, children
