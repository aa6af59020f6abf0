"""Generation step on postfix programs -- test infrastructure.

The paper's loop (sections 1 and 2.1.2) is evaluate -> select -> vary; its
own engine selects on the CPU and varies by mutation only.  The library runs
a classic generational step on the GPU instead: size-t tournament selection,
subtree crossover and point mutation on the reverse-Polish arrays, all driven
by Philox4x32-10 (oracle.philox), and ramped half-and-half initialisation.
This module is the plain reference; the GPU children must equal its output
byte for byte for the same parents, fitness, seed and generation.

Random draws.  Individual c draws 32-bit words from a stream (oracle.philox
.Stream) with counter (c, generation, block, tag): tag = problem id for a
generation step (generation >= 1), tag = 0x80000000 | problem id for
initialisation (generation field 0).  A generation step always reads the
words in this fixed layout, whatever operator it ends up applying:
  j = 0              operator choice            unit(u)
  j = 1 .. t         tournament A entrants      below(u, N)
  j = t+1 .. 2t      tournament B entrants      below(u, N)
  j = 2t+1           crossover point in A       below(u, len A)
  j = 2t+2           crossover point in B       below(u, len B)
  j = 2t+3           mutation position          below(u, len A)
  j = 2t+4           mutation symbol            below(u, choices)
  j = 2t+5           mutation constant          unit(u)
Operator: unit < p_crossover -> crossover; < p_crossover + p_mutation ->
mutation; otherwise a copy of parent A (probabilities and their sum in
binary32).

Tournament: lowest fitness wins, NaN is worse than everything (+Inf
included), ties go to the lowest population index.

A parent that is empty or longer than max_len yields an empty child (the
operators are meant for valid parents; this keeps the result defined).

Subtree crossover: the subtree of postfix token i is the contiguous run
[s, i] whose net stack effect is one value (found by scanning back from i).
Child = A[:sA] + B[sB:iB+1] + A[iA+1:]; a child longer than max_len is
replaced by a copy of A.

Operator sets: op_set 0 uses the nine operators ADD SUB MUL DIV SIN COS EXP
LOG SQRT; op_set 1 the paper's sixteen (its parameter table, section
2.1.7): those nine and SQUARE RECIP TAN ASIN ACOS ATAN TANH, in this order.

Point mutation: the token at the drawn position is replaced by a token of the
same arity, drawn uniformly: binary from (ADD, SUB, MUL, DIV), unary from
the set's unary operators in the order above, terminal from (x_0 .. x_{D-1},
CONST).  A new
CONST gets the value fp32(lo + (hi - lo) * unit) computed in binary64.

Constants: a child's constant table is rebuilt in token order (CONST token
k reads slot k) with the value of the slot it read in its parent; CONST
tokens beyond max_consts become VAR 0.

Microcosm selection (section 2.1.6 of the paper: a sorted random sample of
100 individuals stands in for the ranking of the whole population, and its
percentiles drive one pass of selection that keeps the population at a
target size).  The paper gives no formulas; reading:
  * the sample: draw j of the stream with counter (MICRO_INDEX, generation,
    block, MICRO_TAG | problem) picks individual below(u, N), j = 0 .. s-1
    (with replacement);
  * order: lower fitness first, NaN worse than everything; the sample is
    sorted by (fitness, draw position) and its entry at position
    k = ceil(keep * s) - 1 (clamped to [0, s - 1]) is the threshold tau;
  * survivors: every individual whose fitness is not NaN and <= tau (every
    non-NaN one when tau is NaN), in index order -- one pass; when none
    survives, every individual does;
  * children (any number, so that the population can follow a size
    schedule): child c draws as in the generation step, but parents A and B
    are survivors[below(u_1, S)] and survivors[below(u_{t+1}, S)] (draws
    2..t and t+2..2t are not read), S the number of survivors.  With
    p_crossover = 0 and p_mutation = 1 every child is a point mutant of a
    survivor: the paper's mutation-only variation.

Ramped half-and-half: individual c gets depth d = dmin + (c mod n) with
n = dmax - dmin + 1, and uses the full method when (c div n) is even, grow
otherwise.  Nodes are generated in pre-order: full draws a function
(uniform over the set's F operators, in the order above) above depth d,
grow draws uniformly over the F operators and D+1 terminal symbols, and
level d always draws a terminal
(uniform over D+1 symbols).  A CONST symbol draws its value from the next
word while fewer than max_consts constants exist, else it becomes VAR 0.  The
tree is written in postfix, left operand first.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

from .philox import Stream, below, unit

ADD, SUB, MUL, DIV, SIN, COS, EXP, LOG, SQRT, VAR, CONST = range(11)
SQUARE, RECIP, TAN, ASIN, ACOS, ATAN, TANH = range(11, 18)
BINARY = (ADD, SUB, MUL, DIV)
UNARY = (SIN, COS, EXP, LOG, SQRT)
UNARY_EXT = UNARY + (SQUARE, RECIP, TAN, ASIN, ACOS, ATAN, TANH)
FUNCTIONS = BINARY + UNARY


def unary_set(params) -> tuple:
    return UNARY_EXT if params.op_set == 1 else UNARY


def function_set(params) -> tuple:
    return BINARY + unary_set(params)
INIT_TAG = 0x80000000
MICRO_TAG = 0x40000000
MICRO_INDEX = 0xFFFFFFFF


def arity(op: int) -> int:
    if op in BINARY:
        return 2
    if op in UNARY_EXT:
        return 1
    return 0


@dataclasses.dataclass
class GenParams:
    tournament: int = 4
    p_crossover: float = 0.9
    p_mutation: float = 0.1
    max_len: int = 128
    max_consts: int = 8
    const_lo: float = -5.0
    const_hi: float = 5.0
    init_depth_min: int = 2
    init_depth_max: int = 6
    op_set: int = 0


def const_value(u: int, lo: float, hi: float) -> float:
    """fp32(lo + (hi - lo) * unit(u)), each step rounded in binary64."""
    lo64 = float(np.float32(lo))
    hi64 = float(np.float32(hi))
    span = hi64 - lo64
    prod = span * unit(u)
    return float(np.float32(lo64 + prod))


def operator_thresholds(params: GenParams):
    """Thresholds on unit(u) for crossover and crossover + mutation, in binary32.

    The probabilities are binary32 parameters; the sum is rounded to binary32
    too, and unit(u) is exact in both formats, so the comparisons are exact.
    """
    pc = np.float32(params.p_crossover)
    pm = np.float32(params.p_mutation)
    return float(pc), float(np.float32(pc + pm))


def subtree_start(tokens: Sequence[int], i: int) -> int:
    """Start of the subtree whose root is postfix token i."""
    need = 1
    for j in range(i, -1, -1):
        need += arity(int(tokens[j]) & 0xFF) - 1
        if need == 0:
            return j
    return 0  # malformed parent


def tournament(fitness: np.ndarray, entrants: Sequence[int]) -> int:
    best = None
    for e in entrants:
        f = float(fitness[e])
        key = (1, 0.0, e) if math.isnan(f) else (0, f, e)
        if best is None or key < best:
            best = key
    return best[2]


def renumber(pieces: List[Tuple[int, float]], max_consts: int):
    """pieces: (token, value-if-CONST).  Returns (tokens, consts)."""
    toks: List[int] = []
    consts: List[float] = []
    for t, v in pieces:
        if (t & 0xFF) == CONST:
            if len(consts) < max_consts:
                toks.append(CONST | (len(consts) << 8))
                consts.append(float(np.float32(v)))
            else:
                toks.append(VAR)
        else:
            toks.append(int(t))
    return toks, consts


def _with_values(tokens, consts):
    out = []
    for t in tokens:
        t = int(t)
        if (t & 0xFF) == CONST:
            slot = t >> 8
            out.append((t, float(consts[slot]) if slot < len(consts) else 0.0))
        else:
            out.append((t, 0.0))
    return out


def _sort_key(f: float):
    return (1, 0.0) if math.isnan(f) else (0, f)


def microcosm_threshold(fitness, sample: int, keep: float, seed: int, generation: int, problem: int = 0):
    """tau of the microcosm (NaN when the sample's entry at the keep
    quantile is NaN)."""
    fitness = np.asarray(fitness, dtype=np.float64)
    N = len(fitness)
    s = Stream(seed, MICRO_INDEX, generation, MICRO_TAG | problem)
    drawn = [(float(fitness[below(s.draw(j), N)]), j) for j in range(sample)]
    drawn.sort(key=lambda e: (_sort_key(e[0]), e[1]))
    k = min(sample - 1, max(0, math.ceil(float(np.float32(keep)) * sample) - 1))
    return drawn[k][0]


def survivors(fitness, tau: float) -> List[int]:
    """Indices that survive the threshold, in index order (all when none)."""
    fitness = np.asarray(fitness, dtype=np.float64)
    out = [i for i, f in enumerate(fitness.tolist())
           if not math.isnan(f) and (math.isnan(tau) or f <= tau)]
    return out if out else list(range(len(fitness)))


def make_child(c: int, parents_tok, parents_const, fitness: np.ndarray, D: int,
               params: GenParams, seed: int, generation: int, problem: int = 0, surv=None):
    """(tokens, consts) of child c for one generation step (tournaments, or
    a uniform draw over `surv` for microcosm selection)."""
    N = len(parents_tok)
    t = params.tournament
    s = Stream(seed, c, generation, problem)
    choice = unit(s.draw(0))
    if surv is None:
        ia = tournament(fitness, [below(s.draw(1 + k), N) for k in range(t)])
        ib = tournament(fitness, [below(s.draw(1 + t + k), N) for k in range(t)])
    else:
        ia = surv[below(s.draw(1), len(surv))]
        ib = surv[below(s.draw(1 + t), len(surv))]
    A, Ac = parents_tok[ia], parents_const[ia]
    B, Bc = parents_tok[ib], parents_const[ib]
    LA, LB = len(A), len(B)
    okA = 0 < LA <= params.max_len
    okB = 0 < LB <= params.max_len
    xa = below(s.draw(2 * t + 1), LA if okA else 0)
    xb = below(s.draw(2 * t + 2), LB if okB else 0)
    mpos = below(s.draw(2 * t + 3), LA if okA else 0)
    msym_u = s.draw(2 * t + 4)
    mconst_u = s.draw(2 * t + 5)
    pa = _with_values(A, Ac)
    t_cross, t_mut = operator_thresholds(params)
    if not okA or (choice < t_cross and not okB):
        return [], []
    if choice < t_cross:
        sa = subtree_start(A, xa)
        sb = subtree_start(B, xb)
        pb = _with_values(B, Bc)
        pieces = pa[:sa] + pb[sb:xb + 1] + pa[xa + 1:]
        if len(pieces) > params.max_len:
            pieces = pa
    elif choice < t_mut:
        pieces = list(pa)
        old = int(A[mpos]) & 0xFF
        a = arity(old)
        if a == 2:
            pieces[mpos] = (BINARY[below(msym_u, 4)], 0.0)
        elif a == 1:
            un = unary_set(params)
            pieces[mpos] = (un[below(msym_u, len(un))], 0.0)
        else:
            sym = below(msym_u, D + 1)
            if sym < D:
                pieces[mpos] = (VAR | (sym << 8), 0.0)
            else:
                others = sum(1 for k, (tk, _) in enumerate(pieces)
                             if k != mpos and (tk & 0xFF) == CONST)
                if others < params.max_consts:
                    pieces[mpos] = (CONST, const_value(mconst_u, params.const_lo, params.const_hi))
                else:
                    pieces[mpos] = (VAR, 0.0)
    else:
        pieces = pa
    return renumber(pieces, params.max_consts)


def generation(parents_tok, parents_const, fitness, D: int, params: GenParams,
               seed: int, generation_index: int, problem: int = 0):
    """Children lists (tokens, consts) for every slot c."""
    fitness = np.asarray(fitness, dtype=np.float64)
    return [make_child(c, parents_tok, parents_const, fitness, D, params, seed,
                       generation_index, problem) for c in range(len(parents_tok))]


def generation_microcosm(parents_tok, parents_const, fitness, D: int, params: GenParams, seed: int,
                         generation_index: int, n_children: int, sample: int = 100, keep: float = 0.5,
                         problem: int = 0):
    """Children (tokens, consts) of slots 0 .. n_children - 1 under microcosm selection."""
    fitness = np.asarray(fitness, dtype=np.float64)
    tau = microcosm_threshold(fitness, sample, keep, seed, generation_index, problem)
    surv = survivors(fitness, tau)
    return [make_child(c, parents_tok, parents_const, fitness, D, params, seed, generation_index, problem, surv)
            for c in range(n_children)]


def init_individual(c: int, D: int, params: GenParams, seed: int, problem: int = 0):
    """Ramped half-and-half individual c: (tokens, consts)."""
    n_depths = params.init_depth_max - params.init_depth_min + 1
    depth = params.init_depth_min + (c % n_depths)
    full = ((c // n_depths) % 2) == 0
    s = Stream(seed, c, 0, INIT_TAG | problem)
    cursor = [0]
    toks: List[int] = []
    consts: List[float] = []

    def draw():
        u = s.draw(cursor[0])
        cursor[0] += 1
        return u

    def terminal(sym):
        if sym < D:
            toks.append(VAR | (sym << 8))
        elif len(consts) < params.max_consts:
            toks.append(CONST | (len(consts) << 8))
            consts.append(const_value(draw(), params.const_lo, params.const_hi))
        else:
            toks.append(VAR)

    funcs = function_set(params)

    def node(level):
        if level == depth:
            terminal(below(draw(), D + 1))
            return
        if full:
            op = funcs[below(draw(), len(funcs))]
        else:
            sym = below(draw(), len(funcs) + D + 1)
            if sym >= len(funcs):
                terminal(sym - len(funcs))
                return
            op = funcs[sym]
        for _ in range(arity(op)):
            node(level + 1)
        toks.append(op)

    node(0)
    return toks, consts


def init_population(N: int, D: int, params: GenParams, seed: int, problem: int = 0):
    return [init_individual(c, D, params, seed, problem) for c in range(N)]


def to_fixed(children, max_len: int, max_consts: int):
    """Lists -> the fixed-capacity arrays the library writes (zero padded)."""
    N = len(children)
    tok = np.zeros((N, max_len), dtype=np.uint16)
    ln = np.zeros(N, dtype=np.int32)
    cst = np.zeros((N, max_consts), dtype=np.float32)
    cc = np.zeros(N, dtype=np.int32)
    for c, (t, k) in enumerate(children):
        tok[c, :len(t)] = t
        ln[c] = len(t)
        cst[c, :len(k)] = k
        cc[c] = len(k)
    return tok, ln, cst, cc
