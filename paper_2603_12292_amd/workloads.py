"""Seeded synthetic inputs: postfix program populations and regression datasets.

This module is the one place both sides of every comparison draw their inputs
from (the GPU path and the CPU oracle).  It holds none of the evaluator's
arithmetic: no protected operators, no fitness reductions.  It only

* draws random postfix programs of an exact token length (integers plus fp32
  constants), and
* draws fitness cases X ~ U(lo, hi) and a target y = f(X) for a random target
  expression, evaluated with plain numpy on its natural domain.  A target
  whose evaluation would leave that domain (division by zero, log or sqrt of
  a non-positive number, exp beyond +-80, any non-finite value) is rejected
  and redrawn, so protected-operator conventions never enter the data.

Token encoding (the library's input format, section 2.1.4 of the paper: the
genome is a reverse-Polish program): one uint16 per token,
``opcode | (arg << 8)``; opcodes 0 ADD 1 SUB 2 MUL 3 DIV 4 SIN 5 COS 6 EXP
7 LOG 8 SQRT 9 VAR(arg = variable index) 10 CONST(arg = constant slot).
Binary tokens pop b then a and push ``a op b``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# --- token format -----------------------------------------------------------
ADD, SUB, MUL, DIV, SIN, COS, EXP, LOG, SQRT, VAR, CONST = range(11)
BINARY_OPS = (ADD, SUB, MUL, DIV)
UNARY_OPS = (SIN, COS, EXP, LOG, SQRT)
# the rest of the paper's operator table (unary)
SQUARE, RECIP, TAN, ASIN, ACOS, ATAN, TANH = range(11, 18)
EXTENDED_OPS = (SQUARE, RECIP, TAN, ASIN, ACOS, ATAN, TANH)
OP_NAMES = ("add", "sub", "mul", "div", "sin", "cos", "exp", "log", "sqrt", "var", "const",
            "square", "recip", "tan", "asin", "acos", "atan", "tanh")


def tok(op: int, arg: int = 0) -> int:
    return int(op) | (int(arg) << 8)


def arity_of(op: int) -> int:
    if op in BINARY_OPS:
        return 2
    if op in UNARY_OPS or op in EXTENDED_OPS:
        return 1
    return 0


# --- packed population -------------------------------------------------------
@dataclasses.dataclass
class ProgramSet:
    """A population of postfix programs in the library's packed layout.

    ``tokens[tok_offset[p] : tok_offset[p] + tok_len[p]]`` is program p;
    ``consts[const_offset[p] : const_offset[p] + const_count[p]]`` is its
    constant table (CONST token arg j reads slot j).
    """

    tokens: np.ndarray        # uint16 [n_tokens]
    tok_offset: np.ndarray    # int64 [N]
    tok_len: np.ndarray       # int32 [N]
    consts: np.ndarray        # float32 [n_consts]
    const_offset: np.ndarray  # int64 [N]
    const_count: np.ndarray   # int32 [N]

    @property
    def n(self) -> int:
        return int(self.tok_len.shape[0])

    def program(self, p: int) -> Tuple[np.ndarray, np.ndarray]:
        o, l = int(self.tok_offset[p]), int(self.tok_len[p])
        co, cc = int(self.const_offset[p]), int(self.const_count[p])
        return self.tokens[o:o + l], self.consts[co:co + cc]

    def node_count(self) -> int:
        return int(self.tok_len.astype(np.int64).sum())

    def subset(self, idx: Sequence[int]) -> "ProgramSet":
        return pack_programs([self.program(int(p)) for p in idx])


def pack_programs(progs: Sequence[Tuple[Sequence[int], Sequence[float]]]) -> ProgramSet:
    lens = np.array([len(t) for t, _ in progs], dtype=np.int32)
    ccs = np.array([len(c) for _, c in progs], dtype=np.int32)
    tok_offset = np.zeros(len(progs), dtype=np.int64)
    const_offset = np.zeros(len(progs), dtype=np.int64)
    if len(progs):
        tok_offset[1:] = np.cumsum(lens[:-1], dtype=np.int64)
        const_offset[1:] = np.cumsum(ccs[:-1], dtype=np.int64)
    tokens = np.zeros(int(lens.sum()), dtype=np.uint16)
    consts = np.zeros(int(ccs.sum()), dtype=np.float32)
    for p, (t, c) in enumerate(progs):
        tokens[tok_offset[p]:tok_offset[p] + lens[p]] = np.asarray(t, dtype=np.uint16)
        consts[const_offset[p]:const_offset[p] + ccs[p]] = np.asarray(c, dtype=np.float32)
    return ProgramSet(tokens, tok_offset, lens, consts, const_offset, ccs)


# --- random programs of an exact length ---------------------------------------
def random_program(rng: np.random.Generator, length: int, D: int, *, max_consts: int = 8,
                   const_lo: float = -5.0, const_hi: float = 5.0,
                   allow_const: bool = True, unary=None) -> Tuple[List[int], List[float]]:
    """One valid postfix program of exactly ``length`` tokens.

    Left to right, each token is drawn uniformly among the symbols that still
    let the program close to a single value in the tokens that remain: the
    four binary operators (need two values on the stack), the unary ones
    (need one; the five of the base set, or the opcodes in ``unary``) and
    the D+1 terminal symbols x_0..x_{D-1}, CONST (allowed while
    depth + 1 <= tokens remaining).  CONST draws beyond ``max_consts`` become
    x_0.  Constants are U(const_lo, const_hi) rounded to fp32.
    """
    unary_ops = UNARY_OPS if unary is None else tuple(unary)
    if length < 1:
        raise ValueError("length must be >= 1")
    toks: List[int] = []
    consts: List[float] = []
    depth = 0
    n_term_syms = D + (1 if allow_const else 0)
    for pos in range(length):
        # After this token r tokens remain; a stack of depth d' >= 1 can close
        # to one value in exactly r tokens iff d' - 1 <= r (d' - 1 binaries,
        # the rest filled with unary operators).
        r = length - pos - 1
        ok: List[Tuple[int, int]] = []   # (kind, symbol)
        if depth + 1 - 1 <= r:
            ok += [(0, s) for s in range(n_term_syms)]
        if depth >= 1 and depth - 1 <= r:
            ok += [(1, op) for op in unary_ops]
        if depth >= 2 and depth - 2 <= r:
            ok += [(2, op) for op in BINARY_OPS]
        kind, sym = ok[int(rng.integers(len(ok)))]
        if kind == 0:
            if sym == D:  # CONST
                if len(consts) < max_consts:
                    toks.append(tok(CONST, len(consts)))
                    consts.append(float(np.float32(rng.uniform(const_lo, const_hi))))
                else:
                    toks.append(tok(VAR, 0))
            else:
                toks.append(tok(VAR, sym))
            depth += 1
        elif kind == 1:
            toks.append(tok(sym))
        else:
            toks.append(tok(sym))
            depth -= 1
    assert depth == 1, (toks, depth)
    return toks, consts


def place_constants(rng: np.random.Generator, toks: List[int], k: int, *,
                    const_lo: float = -5.0, const_hi: float = 5.0) -> Tuple[List[int], List[float]]:
    """Turn k of a program's terminals (chosen uniformly) into CONST slots 0..k-1."""
    term_pos = [i for i, t in enumerate(toks) if (t & 0xFF) in (VAR, CONST)]
    k = min(k, len(term_pos))
    chosen = sorted(rng.choice(len(term_pos), size=k, replace=False).tolist())
    out = list(toks)
    consts: List[float] = []
    for j, ti in enumerate(sorted(term_pos[c] for c in chosen)):
        out[ti] = tok(CONST, j)
        consts.append(float(np.float32(rng.uniform(const_lo, const_hi))))
    return out, consts


def random_population(seed: int, N: int, len_lo: int, len_hi: int, D: int, *,
                      max_consts: int = 8, const_range: Tuple[float, float] = (-5.0, 5.0),
                      consts_per_program: Optional[Tuple[int, int]] = None, unary=None) -> ProgramSet:
    """N programs, lengths uniform on {len_lo..len_hi}.

    With ``consts_per_program=(a, b)`` each program first gets a variables-only
    skeleton, then k ~ U{a..b} of its terminals become constants.  ``unary``:
    the unary opcodes to draw from (default: the five of the base set).
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5052]))
    progs = []
    lo, hi = const_range
    for _ in range(N):
        L = int(rng.integers(len_lo, len_hi + 1))
        if consts_per_program is None:
            progs.append(random_program(rng, L, D, max_consts=max_consts, const_lo=lo, const_hi=hi, unary=unary))
        else:
            t, _ = random_program(rng, L, D, allow_const=False, unary=unary)
            k = int(rng.integers(consts_per_program[0], consts_per_program[1] + 1))
            progs.append(place_constants(rng, t, k, const_lo=lo, const_hi=hi))
    return pack_programs(progs)


# --- target expressions on their natural domain --------------------------------
class _DomainError(Exception):
    pass


def _target_value(toks: Sequence[int], consts: Sequence[float], X64: np.ndarray) -> np.ndarray:
    """Evaluate a target expression with plain numpy math (float64).

    Builds the expression tree from the postfix tokens, then evaluates it
    recursively.  Raises _DomainError where a plain operator is undefined.
    """
    nodes = []
    for t in toks:
        op, arg = t & 0xFF, t >> 8
        a = arity_of(op)
        kids = [nodes.pop() for _ in range(a)][::-1]
        nodes.append((op, arg, kids))
    (root,) = nodes

    def ev(node):
        op, arg, kids = node
        if op == VAR:
            return X64[:, arg]
        if op == CONST:
            return np.full(X64.shape[0], float(consts[arg]))
        v = [ev(k) for k in kids]
        with np.errstate(all="raise"):
            try:
                if op == ADD:
                    r = v[0] + v[1]
                elif op == SUB:
                    r = v[0] - v[1]
                elif op == MUL:
                    r = v[0] * v[1]
                elif op == DIV:
                    if np.any(v[1] == 0):
                        raise _DomainError
                    r = v[0] / v[1]
                elif op == SIN:
                    r = np.sin(v[0])
                elif op == COS:
                    r = np.cos(v[0])
                elif op == EXP:
                    if np.any(np.abs(v[0]) > 80):
                        raise _DomainError
                    r = np.exp(v[0])
                elif op == LOG:
                    if np.any(v[0] <= 0):
                        raise _DomainError
                    r = np.log(v[0])
                elif op == SQRT:
                    if np.any(v[0] < 0):
                        raise _DomainError
                    r = np.sqrt(v[0])
                else:
                    raise ValueError(op)
            except FloatingPointError:
                raise _DomainError
        if not np.all(np.isfinite(r)):
            raise _DomainError
        return r

    return ev(root)


@dataclasses.dataclass
class Dataset:
    X: np.ndarray            # float32 [M, D], row-major (case-major)
    y: np.ndarray            # float32 [M]
    target_tokens: List[int]
    target_consts: List[float]

    @property
    def M(self) -> int:
        return int(self.X.shape[0])

    @property
    def D(self) -> int:
        return int(self.X.shape[1])


def make_dataset(seed: int, M: int, D: int, *, x_range=(1.0, 5.0), target_len: int = 10,
                 noise: float = 0.0) -> Dataset:
    """Fitness cases X ~ U(x_range) (fp32) and y = target(X) [+ noise].

    The target is a random ``target_len``-token expression that uses at least
    one variable, stays on its natural domain over all M cases and is not
    near-constant (std(y) >= 1e-6 * rms(y)).  ``noise`` adds Gaussian noise
    with standard deviation ``noise * rms(y)``.
    """
    ss = np.random.SeedSequence([seed, 0xDA7A])
    s_x, s_t, s_n = ss.spawn(3)
    X = np.random.default_rng(s_x).uniform(x_range[0], x_range[1], size=(M, D)).astype(np.float32)
    X64 = X.astype(np.float64)
    rng_t = np.random.default_rng(s_t)
    for _attempt in range(100000):
        toks, consts = random_program(rng_t, target_len, D)
        if not any((t & 0xFF) == VAR for t in toks):
            continue
        try:
            y64 = _target_value(toks, consts, X64)
        except _DomainError:
            continue
        rms = math.sqrt(float(np.mean(y64 * y64)))
        if not (rms > 0 and np.std(y64) >= 1e-6 * rms):
            continue
        if np.max(np.abs(y64)) > 1e30:
            continue
        if noise > 0:
            y64 = y64 + np.random.default_rng(s_n).normal(0.0, noise * rms, size=M)
        y = y64.astype(np.float32)
        if not np.all(np.isfinite(y)):
            continue
        return Dataset(X, y, toks, consts)
    raise RuntimeError("no admissible target expression found")


# --- the configurations ------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    programs: ProgramSet
    data: Dataset


def replicate(ps: "ProgramSet", times: int) -> "ProgramSet":
    """The population repeated `times` times, every copy with its own token
    and constant storage (program p of copy r is program r * n + p)."""
    n_tok = int(ps.tokens.shape[0])
    n_const = int(ps.consts.shape[0])
    reps = np.arange(times, dtype=np.int64)
    return ProgramSet(
        tokens=np.tile(ps.tokens, times),
        tok_offset=(ps.tok_offset[None, :] + reps[:, None] * n_tok).reshape(-1).astype(np.int64),
        tok_len=np.tile(ps.tok_len, times),
        consts=np.tile(ps.consts, times),
        const_offset=(ps.const_offset[None, :] + reps[:, None] * n_const).reshape(-1).astype(np.int64),
        const_count=np.tile(ps.const_count, times),
    )


def config_paper_shape(seed: int = 2611, *, copies: int = 256, M: int = 512) -> Workload:
    """The paper's regime (about 10^6 individuals, 512 fitness cases per
    generation): the plain-mid population (N = 4096, L ~ U{5..64}, D = 5)
    replicated to 2^20 programs, on 512 cases drawn like plain-mid's."""
    base = config_mid()
    data = make_dataset(seed, M, 5, x_range=(1.0, 10.0), target_len=20)
    return Workload(f"paper-shape: N={base.programs.n * copies} (plain-mid x{copies}), L~U{{5..64}}, D=5, M={M}",
                    replicate(base.programs, copies), data)


def invalid_target_dataset(seed: int, M: int, D: int, *, x_range=(1.0, 5.0)) -> Dataset:
    """Targets undefined on part of the domain, as the paper's scores are
    built for: y = log(x0 - 2) * (1 + x1 / 4) evaluated in binary64 without
    protection (NaN where x0 < 2), rounded to binary32; X ~ U(x_range)."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(x_range[0], x_range[1], size=(M, D)).astype(np.float32)
    X64 = X.astype(np.float64)
    x1 = X64[:, 1] if D > 1 else X64[:, 0]
    with np.errstate(invalid="ignore", divide="ignore"):
        y = (np.log(X64[:, 0] - 2.0) * (1.0 + x1 / 4.0)).astype(np.float32)
    return Dataset(X, y, [], [])


def config_tiny(seed: int = 2604) -> Workload:
    """N=256, L~U{3..32}, D=3, M=1000, X~U(1,5), 10-token target + 1% noise."""
    progs = random_population(seed, 256, 3, 32, 3)
    data = make_dataset(seed, 1000, 3, x_range=(1.0, 5.0), target_len=10, noise=0.01)
    return Workload("plain-tiny N=256 L=3..32 D=3 M=1000", progs, data)


def config_mid(seed: int = 2605, *, N: int = 4096, M: int = 100_000) -> Workload:
    """N=4096, L~U{5..64}, <=8 consts, D=5, M=100000, X~U(1,10), 20-token target."""
    progs = random_population(seed, N, 5, 64, 5)
    data = make_dataset(seed, M, 5, x_range=(1.0, 10.0), target_len=20)
    return Workload(f"plain-mid N={N} L=5..64 D=5 M={M}", progs, data)


def config_differentiation(seed: int = 2608, *, N: int = 4096, M: int = 100_000) -> Workload:
    """N=4096 programs with 1..8 constants, L~U{8..64}, D=5, M=100000 (data as plain-mid)."""
    progs = random_population(seed, N, 8, 64, 5, consts_per_program=(1, 8))
    data = make_dataset(seed, M, 5, x_range=(1.0, 10.0), target_len=20)
    return Workload(f"adjoint N={N} L=8..64 consts=1..8 D=5 M={M}", progs, data)


def generation_dataset(seed: int = 2606, *, M: int = 1_000_000, D: int = 9) -> Dataset:
    """Data of the generation-loop workload: D=9, M=1e6, X~U(1,5), 30-token target."""
    return make_dataset(seed, M, D, x_range=(1.0, 5.0), target_len=30)


def ragged_problems(seed: int = 2607, *, n_problems: int = 64, n_programs: int = 1024,
                    len_lo: int = 5, len_hi: int = 96, m_lo: float = 1e3, m_hi: float = 1e6,
                    d_lo: int = 1, d_hi: int = 9) -> List[Workload]:
    """Independent regression problems of the ragged-batching workload.

    Per problem: D ~ U{d_lo..d_hi}, M = round(10**U(log10 m_lo, log10 m_hi)),
    X ~ U(1,5), 10-token target + 1% noise, n_programs programs of
    L ~ U{len_lo..len_hi}.
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xBA7C]))
    out = []
    for q in range(n_problems):
        D = int(rng.integers(d_lo, d_hi + 1))
        M = int(round(10 ** rng.uniform(math.log10(m_lo), math.log10(m_hi))))
        progs = random_population(seed * 1000 + q, n_programs, len_lo, len_hi, D)
        data = make_dataset(seed * 1000 + q, M, D, x_range=(1.0, 5.0), target_len=10, noise=0.01)
        out.append(Workload(f"ragged[{q}] D={D} M={M}", progs, data))
    return out
