"""Readable program notation for tests: 'x0 x1 + c0 *' -> uint16 token list."""
import numpy as np

_OPS = {"+": 0, "-": 1, "*": 2, "/": 3, "sin": 4, "cos": 5, "exp": 6, "log": 7, "sqrt": 8,
        "sq": 11, "inv": 12, "tan": 13, "asin": 14, "acos": 15, "atan": 16, "tanh": 17}
_NAMES = {v: k for k, v in _OPS.items()}


def parse(text):
    out = []
    for w in text.split():
        if w in _OPS:
            out.append(_OPS[w])
        elif w[0] == "x":
            out.append(9 | (int(w[1:]) << 8))
        elif w[0] == "c":
            out.append(10 | (int(w[1:]) << 8))
        else:
            raise ValueError(w)
    return out


def show(tokens):
    out = []
    for t in tokens:
        op, arg = int(t) & 0xFF, int(t) >> 8
        if op == 9:
            out.append(f"x{arg}")
        elif op == 10:
            out.append(f"c{arg}")
        else:
            out.append(_NAMES.get(op, f"?{op}"))
    return " ".join(out)


def same(a, b):
    """Bitwise-equal float64 arrays, all NaNs considered equal."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    both_nan = np.isnan(a) & np.isnan(b)
    return bool(np.all(both_nan | (a.view(np.uint64) == b.view(np.uint64))))
