"""Pins of the oracle's stack interpreter (CPU only)."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import interp, tree
from progtext import parse, same, show

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _hand_cases():
    cases = []
    with open(os.path.join(GOLDEN, "hand_expressions.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            prog, consts, xs, expected = [p.strip() for p in line.split(";")]
            cases.append((prog, [float(v) for v in consts.split()], [float(v) for v in xs.split()],
                          eval(expected, {"math": math})))
    return cases


@pytest.mark.parametrize("prog,consts,xs,expected", _hand_cases())
def test_hand_evaluated(prog, consts, xs, expected):
    toks = parse(prog)
    X = np.array([xs], dtype=np.float32)
    got = interp.run(toks, consts, X, "o64")[0]
    assert got == pytest.approx(expected, rel=1e-15, abs=0)
    # o32e is the same value rounded after every token
    got32 = interp.run(toks, consts, X, "o32e")[0]
    if math.isfinite(expected) and abs(expected) < 3e38:
        assert got32 == pytest.approx(expected, rel=2e-6)


# special values: (op, inputs, expected) for both modes; derived from the
# operator conventions written in oracle/interp.py's header
INF = math.inf
NAN = math.nan
DEN = float(np.float32(1e-40))   # a binary32 denormal
SPECIAL = [
    ("/", (1.0, 0.0), 1.0), ("/", (1.0, -0.0), 1.0), ("/", (NAN, 0.0), 1.0),
    ("/", (1.0, NAN), NAN), ("/", (1.0, INF), 0.0), ("/", (-1.0, INF), -0.0),
    ("/", (INF, INF), NAN), ("/", (INF, 2.0), INF), ("/", (0.0, 0.0), 1.0),
    ("sin", (INF,), NAN), ("sin", (-INF,), NAN), ("sin", (NAN,), NAN), ("sin", (-0.0,), -0.0),
    ("cos", (INF,), NAN), ("cos", (-INF,), NAN), ("cos", (NAN,), NAN),
    ("exp", (INF,), math.exp(80.0)), ("exp", (-INF,), math.exp(-80.0)), ("exp", (NAN,), NAN),
    ("exp", (80.0,), math.exp(80.0)), ("exp", (-80.0,), math.exp(-80.0)),
    ("exp", (0.0,), 1.0), ("exp", (DEN,), 1.0),
    ("log", (0.0,), 0.0), ("log", (-0.0,), 0.0), ("log", (INF,), INF), ("log", (-INF,), INF),
    ("log", (NAN,), NAN), ("log", (-1.0,), 0.0), ("log", (DEN,), math.log(DEN)),
    ("sqrt", (-4.0,), 2.0), ("sqrt", (-INF,), INF), ("sqrt", (INF,), INF), ("sqrt", (NAN,), NAN),
    ("sqrt", (-0.0,), 0.0), ("sqrt", (DEN,), math.sqrt(DEN)),
    ("+", (INF, -INF), NAN), ("*", (0.0, INF), NAN), ("-", (INF, INF), NAN),
]


@pytest.mark.parametrize("op,args,expected", SPECIAL)
def test_special_values(op, args, expected):
    if len(args) == 2:
        toks = parse(f"x0 x1 {op}")
    else:
        toks = parse(f"x0 {op}")
    X = np.array([list(args) + [0.0] * (2 - len(args))], dtype=np.float32)
    for mode in ("o64", "o32e"):
        got = interp.run(toks, [], X, mode)[0]
        exp = expected if mode == "o64" else float(np.float32(expected))
        if math.isnan(exp):
            assert math.isnan(got), (op, args, mode, got)
        elif exp == 0.0:
            assert got == 0.0 and math.copysign(1, got) == math.copysign(1, exp), (op, args, mode, got)
        else:
            assert got == pytest.approx(exp, rel=1e-15), (op, args, mode, got)
        # the tree evaluator agrees
        tv = tree.run(toks, [], X, round32=(mode == "o32e"))[0]
        assert same([got], [tv])


def _all_programs(max_len, symbols, arity):
    """Every valid postfix sequence of length 1..max_len over the symbols."""
    for L in range(1, max_len + 1):
        for seq in itertools.product(symbols, repeat=L):
            d = 0
            ok = True
            for s in seq:
                a = arity[s]
                if d < a:
                    ok = False
                    break
                d += 1 - a
            if ok and d == 1:
                yield list(seq)


_SYMS = [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 9 | 256, 10, 10 | 256]
_AR = {s: (2 if (s & 0xFF) < 4 else 1 if (s & 0xFF) < 9 else 0) for s in _SYMS}
_ROWS = np.array([[2.0, 3.0], [0.0, -1.5], [-0.0, 0.0], [1e30, -1e-30], [90.0, -90.0],
                  [float(np.float32(1e-40)), 7.0], [np.inf, 2.0], [np.nan, 1.0]], dtype=np.float32)
_CONSTS = [0.5, -2.25]


def test_bruteforce_against_tree_evaluator():
    """All valid programs of <= 5 tokens (D=2, two constants, 9 operators),
    bit for bit in both modes, on rows holding special values."""
    n = 0
    for toks in _all_programs(5, _SYMS, _AR):
        st, _ = interp.validate(toks, 2, 2)
        assert st == interp.ST_OK
        for mode, r32 in (("o64", False), ("o32e", True)):
            a = interp.run(toks, _CONSTS, _ROWS, mode)
            b = tree.run(toks, _CONSTS, _ROWS, round32=r32)
            assert same(a, b), (show(toks), mode, a, b)
        n += 1
    assert n > 15000


def test_random_programs_against_tree_evaluator():
    from paper_2603_12292_amd.workloads import random_program
    rng = np.random.default_rng(12345)
    X = rng.uniform(-3, 3, size=(16, 3)).astype(np.float32)
    for _ in range(2000):
        L = int(rng.integers(1, 40))
        toks, consts = random_program(rng, L, 3)
        for mode, r32 in (("o64", False), ("o32e", True)):
            a = interp.run(toks, consts, X, mode)
            b = tree.run(toks, consts, X, round32=r32)
            assert same(a, b), (show(toks), mode)


def test_o32e_matches_ieee_binary32():
    """Rounding every token's binary64 result gives IEEE fp32 for + - * / sqrt."""
    rng = np.random.default_rng(7)
    n = 200_000
    a = (rng.standard_normal(n) * np.exp(rng.uniform(-80, 80, n))).astype(np.float32)
    b = (rng.standard_normal(n) * np.exp(rng.uniform(-80, 80, n))).astype(np.float32)
    edge = np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, np.nan, 1e-45, -1e-45, 3.4028235e38,
                     -3.4028235e38, 1.1754944e-38, 1e-40, 16777217.0], dtype=np.float32)
    ea, eb = np.meshgrid(edge, edge)
    a = np.concatenate([a, ea.ravel()])
    b = np.concatenate([b, eb.ravel()]).astype(np.float32)
    X = np.stack([a, b], axis=1)
    with np.errstate(all="ignore"):
        ref = {"+": a + b, "-": a - b, "*": a * b,
               "/": np.where(b == 0, np.float32(1), a / np.where(b == 0, np.float32(1), b)),
               "sqrt": np.sqrt(np.abs(a))}
    for op, r in ref.items():
        toks = parse("x0 sqrt" if op == "sqrt" else f"x0 x1 {op}")
        got = interp.run(toks, [], X, "o32e")
        assert same(got, r.astype(np.float64)), op


BAD = [
    ("", 0, 2, interp.ST_EMPTY),
    ("x0 +", 0, 2, interp.ST_UNDERFLOW),
    ("sin", 0, 2, interp.ST_UNDERFLOW),
    ("x0 x1", 0, 2, interp.ST_BAD_FINAL_DEPTH),
    ("x2", 0, 2, interp.ST_BAD_VAR),
    ("c0", 0, 2, interp.ST_BAD_CONST),
    ("c1", 1, 2, interp.ST_BAD_CONST),
    ("x0 c0 +", 1, 2, interp.ST_OK),
    ("x0 x1 + x0", 0, 2, interp.ST_BAD_FINAL_DEPTH),
]


@pytest.mark.parametrize("prog,cc,D,status", BAD)
def test_validate(prog, cc, D, status):
    assert interp.validate(parse(prog), cc, D)[0] == status


def test_validate_opcode_and_priority():
    assert interp.validate([18], 0, 1)[0] == interp.ST_BAD_OPCODE
    assert interp.validate([9, 17], 0, 1) == (interp.ST_OK, 1)  # TANH: the last opcode
    assert interp.validate([9, 0xFF], 0, 1)[0] == interp.ST_BAD_OPCODE
    # first faulty token decides: bad var before a later underflow
    assert interp.validate(parse("x5 +"), 0, 2)[0] == interp.ST_BAD_VAR
    assert interp.validate(parse("+ x5"), 0, 2)[0] == interp.ST_UNDERFLOW
    assert interp.validate([9] * 4097, 0, 1)[0] == interp.ST_TOO_LONG
    assert interp.validate(parse("x0 x1 x0 * +"), 0, 2) == (interp.ST_OK, 3)


def test_o32p_perturbs_only_non_arithmetic_operators():
    rng = np.random.default_rng(3)
    X = rng.uniform(1, 5, size=(200, 2)).astype(np.float32)
    toks = parse("x0 x1 / x0 x1 * * x1 -")
    assert same(interp.run(toks, [], X, "o32p", seed=4), interp.run(toks, [], X, "o32e"))
    assert not same(interp.run(parse("x0 x1 + sqrt"), [], X, "o32p", seed=4),
                    interp.run(parse("x0 x1 + sqrt"), [], X, "o32e"))
    toks = parse("x0 sin x1 exp *")
    a = interp.run(toks, [], X, "o32p", seed=4)
    b = interp.run(toks, [], X, "o32e")
    assert not same(a, b)
    assert np.all(np.abs(a - b) <= 2 ** -20 * np.abs(b))
    assert same(a, interp.run(toks, [], X, "o32p", seed=4))



# ---- the paper's further operators (SQUARE RECIP TAN ASIN ACOS ATAN TANH)

def test_extended_special_values():
    X = np.array([[3.0], [0.0], [-0.0], [2.0], [-1.0], [1.0], [np.inf], [np.nan]], dtype=np.float32)
    r = {name: interp.run(parse(f"x0 {name}"), [], X) for name in ("sq", "inv", "tan", "asin", "acos", "atan", "tanh")}
    assert r["sq"][0] == 9.0 and r["inv"][0] == 1.0 / 3.0
    assert r["inv"][1] == math.inf and r["inv"][2] == -math.inf          # 1/x at +-0
    assert math.isnan(r["asin"][3]) and math.isnan(r["acos"][3])         # outside [-1, 1]
    assert r["acos"][4] == math.pi and r["asin"][5] == math.pi / 2 and r["acos"][5] == 0.0
    assert math.isnan(r["tan"][6]) and r["atan"][6] == math.pi / 2 and r["tanh"][6] == 1.0
    assert all(math.isnan(v[7]) for v in r.values())
    assert r["tanh"][1] == 0.0 and r["atan"][1] == 0.0 and r["tan"][1] == 0.0


def test_extended_identities():
    """Inverse pairs and the defining formulas of the further operators,
    each written as a program over the base operators where one exists."""
    rng = np.random.default_rng(7)
    X = np.stack([rng.uniform(-0.99, 0.99, 500), rng.uniform(-1.5, 1.5, 500)], axis=1).astype(np.float32)
    x = X[:, 0].astype(np.float64)
    t = X[:, 1].astype(np.float64)
    run = lambda prog, c=(): interp.run(parse(prog), list(c), X)
    assert np.allclose(run("x0 asin sin"), x, rtol=0, atol=1e-15)
    assert np.allclose(run("x0 acos cos"), x, rtol=0, atol=1e-15)
    assert np.allclose(run("x0 asin x0 acos +"), np.full(500, math.pi / 2), rtol=0, atol=1e-15)
    assert np.allclose(run("x1 atan tan"), t, rtol=0, atol=1e-15)
    # tan = sin / cos, square = x * x exactly, 1 / (1 / x) = x
    assert np.allclose(run("x1 tan"), run("x1 sin x1 cos /"), rtol=1e-15, atol=0)
    assert np.array_equal(run("x1 sq"), run("x1 x1 *"))
    assert np.allclose(run("x1 inv inv"), t, rtol=2e-16, atol=0)
    # tanh x = (e^2x - 1) / (e^2x + 1)
    assert np.allclose(run("x1 tanh"), run("x1 x1 + exp c0 - x1 x1 + exp c0 + /", [1.0]), rtol=1e-15, atol=1e-16)


def test_extended_against_tree_evaluator():
    """Random programs over all twelve unary operators, both modes, bit for
    bit against the tree evaluator (including NaN and Inf outputs)."""
    from paper_2603_12292_amd.workloads import random_program
    rng = np.random.default_rng(54321)
    X = np.concatenate([rng.uniform(-3, 3, size=(14, 3)), [[0.0, -0.0, 1.0], [np.inf, 0.5, -1.0]]]).astype(np.float32)
    un = (4, 5, 6, 7, 8) + tuple(range(11, 18))
    n_ext = 0
    for _ in range(1500):
        toks, consts = random_program(rng, int(rng.integers(1, 30)), 3, unary=un)
        n_ext += any((t & 0xFF) >= 11 for t in toks)
        for mode, r32 in (("o64", False), ("o32e", True)):
            a = interp.run(toks, consts, X, mode)
            b = tree.run(toks, consts, X, round32=r32)
            assert same(a, b), (show(toks), mode)
    assert n_ext > 800


def test_extended_o32e_exact_operators():
    """SQUARE and RECIP rounded once equal IEEE binary32 x * x and 1 / x."""
    rng = np.random.default_rng(9)
    x = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-20, 20, 2000),
                        [0.0, -0.0, 1e-45, 3e38]]).astype(np.float32)
    X = x[:, None]
    with np.errstate(all="ignore"):
        assert same(interp.run(parse("x0 sq"), [], X, "o32e"), (x * x).astype(np.float64))
        assert same(interp.run(parse("x0 inv"), [], X, "o32e"), (np.float32(1.0) / x).astype(np.float64))
