"""Independent recursive tree evaluator -- test infrastructure.

A second reading of the same reverse-Polish programs (paper, section 2.1.4):
the postfix tokens are parsed into an explicit expression tree, which is then
evaluated case by case with scalar Python arithmetic.  It shares no code with
``oracle.interp`` (explicit tree instead of a value stack, one case at a time
instead of whole vectors), so agreement between the two pins operand order,
arity handling and the operator conventions.  The elementary functions sin,
cos, exp and log are taken from numpy (called on one-element arrays, which
numpy evaluates exactly as it does inside longer arrays) so that the two
evaluators can be compared bit for bit; so are tan, asin, acos, atan and
tanh, with their domain rules (NaN outside [-1, 1] for asin and acos, NaN
for tan of +-Inf) and 1/x at +-0 (+-Inf) written out here.
"""
from __future__ import annotations

import math

import numpy as np

_NAMES = {0: "+", 1: "-", 2: "*", 3: "/", 4: "sin", 5: "cos", 6: "exp", 7: "log", 8: "sqrt",
          11: "sq", 12: "inv", 13: "tan", 14: "asin", 15: "acos", 16: "atan", 17: "tanh"}
_UNARY = (4, 5, 6, 7, 8, 11, 12, 13, 14, 15, 16, 17)


class Node:
    __slots__ = ("kind", "arg", "kids", "pos")

    def __init__(self, kind, arg, kids, pos=-1):
        self.kind = kind
        self.arg = arg
        self.kids = kids
        self.pos = pos  # index of the node's token in the postfix program


def parse(tokens) -> Node:
    """Postfix tokens -> expression tree (raises on malformed programs)."""
    st = []
    for i, t in enumerate(tokens):
        op, arg = int(t) & 0xFF, int(t) >> 8
        if op == 9:
            st.append(Node("var", arg, [], i))
        elif op == 10:
            st.append(Node("const", arg, [], i))
        elif op in (0, 1, 2, 3):
            right = st.pop()
            left = st.pop()
            st.append(Node(_NAMES[op], 0, [left, right], i))
        elif op in _UNARY:
            st.append(Node(_NAMES[op], 0, [st.pop()], i))
        else:
            raise ValueError(op)
    if len(st) != 1:
        raise ValueError("program does not reduce to one value")
    return st[0]


def to_postfix(node: Node):
    """Serialise a tree back to tokens (left subtree first)."""
    codes = {v: k for k, v in _NAMES.items()}
    out = []

    def walk(n):
        for k in n.kids:
            walk(k)
        if n.kind == "var":
            out.append(9 | (n.arg << 8))
        elif n.kind == "const":
            out.append(10 | (n.arg << 8))
        else:
            out.append(codes[n.kind])

    walk(node)
    return out


def size(node: Node) -> int:
    return 1 + sum(size(k) for k in node.kids)


def _r32(v: float) -> float:
    with np.errstate(over="ignore"):
        return float(np.float32(v))


def _np1(f, x: float) -> float:
    with np.errstate(all="ignore"):
        return float(f(np.array([x], dtype=np.float64))[0])


def _scalar(kind, vals):
    if kind == "+":
        return vals[0] + vals[1]
    if kind == "-":
        return vals[0] - vals[1]
    if kind == "*":
        return vals[0] * vals[1]
    if kind == "/":
        a, b = vals
        if b == 0.0:
            return 1.0
        return a / b
    x = vals[0]
    if kind in ("sin", "cos"):
        if math.isinf(x):
            return math.nan
        return _np1(np.sin if kind == "sin" else np.cos, x)
    if kind == "exp":
        if x > 80.0:
            x = 80.0
        elif x < -80.0:
            x = -80.0
        return _np1(np.exp, x)  # NaN stays NaN
    if kind == "log":
        if x == 0.0:
            return 0.0
        if math.isnan(x):
            return math.nan
        return _np1(np.log, abs(x))
    if kind == "sqrt":
        return math.sqrt(abs(x))
    if kind == "sq":
        return x * x
    if kind == "inv":
        if x == 0.0:
            return math.copysign(math.inf, x)
        return 1.0 / x
    if kind == "tan":
        return math.nan if math.isinf(x) else _np1(np.tan, x)
    if kind in ("asin", "acos"):
        if not abs(x) <= 1.0:
            return math.nan
        return _np1(np.arcsin if kind == "asin" else np.arccos, x)
    if kind == "atan":
        return _np1(np.arctan, x)
    if kind == "tanh":
        return _np1(np.tanh, x)
    raise ValueError(kind)


def evaluate(node: Node, xrow, consts, round32: bool = False, perturb=None, row: int = 0) -> float:
    """Value of the tree for one fitness case (a row of X).

    ``perturb(pos, row, v)``, when given, replaces the result v of every
    operator node (token index pos) before its parent uses it: a way to
    impose chosen errors on chosen operations, case by case.
    """
    if node.kind == "var":
        return float(xrow[node.arg])
    if node.kind == "const":
        return float(consts[node.arg])
    v = _scalar(node.kind, [evaluate(k, xrow, consts, round32, perturb, row) for k in node.kids])
    if perturb is not None:
        v = perturb(node.pos, row, v)
    return _r32(v) if round32 else v


def run(tokens, consts, X, round32: bool = False, perturb=None) -> np.ndarray:
    root = parse(tokens)
    c = [float(np.float32(v)) for v in consts]
    Xf = np.asarray(X, dtype=np.float32)
    return np.array([evaluate(root, [float(v) for v in row], c, round32, perturb, i) for i, row in enumerate(Xf)])
