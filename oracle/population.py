"""Whole-population evaluation -> fitness[N] -- test infrastructure.

Section 2.1.2 of the paper: every genome of the population is run on a batch
of fitness cases and one aggregate fitness per individual comes back.  This
module loops over programs (validate, interpret, reduce) in the plainest way;
``processes > 1`` splits the program list over a process pool (one
single-threaded worker per core) for the CPU-baseline timing.
"""
from __future__ import annotations

import math
import os
import sys
from typing import Optional

import numpy as np

from . import bound as obound
from . import fitness as fit
from . import interp


def program_slices(tok_offset, tok_len, const_offset, const_count):
    for p in range(len(tok_len)):
        yield (int(tok_offset[p]), int(tok_len[p]), int(const_offset[p]), int(const_count[p]))


def evaluate_one(tokens, consts, X, y, kind: int, mode: str = "o64", seed: int = 0):
    """(fitness, status) of one program."""
    D = X.shape[1]
    st, _ = interp.validate(tokens, len(consts), D)
    if st != interp.ST_OK:
        return math.nan, st
    yh = interp.run(tokens, consts, X, mode, seed)
    return fit.fitness(kind, yh, y), st


def bound_one(tokens, consts, X, y, kind: int, div_eps=None):
    """(first-order fitness bound of oracle.bound, status) of one program;
    NaN for an invalid program."""
    st, _ = interp.validate(tokens, len(consts), X.shape[1])
    if st != interp.ST_OK:
        return math.nan, st
    return obound.fitness_bound(tokens, consts, X, y, kind, div_eps=div_eps), st


def _worker(args):
    tokens, consts, tok_offset, tok_len, const_offset, const_count, X, y, kind, mode, lo, hi, seed, div_eps = args
    out = np.empty(hi - lo)
    sts = np.empty(hi - lo, dtype=np.int8)
    for i, p in enumerate(range(lo, hi)):
        o, l = int(tok_offset[p]), int(tok_len[p])
        co, cc = int(const_offset[p]), int(const_count[p])
        if mode == "bound":
            out[i], sts[i] = bound_one(tokens[o:o + l], consts[co:co + cc], X, y, kind, div_eps)
        else:
            out[i], sts[i] = evaluate_one(tokens[o:o + l], consts[co:co + cc], X, y, kind, mode,
                                          seed * 1_000_003 + p)
    return lo, out, sts


def _gpu_runtime_started() -> bool:
    """Whether this process has initialised a GPU runtime (through torch):
    its threads make fork() unsafe (a forked child can block forever on a
    lock one of them held), so the pool is not used then."""
    torch = sys.modules.get("torch")
    try:
        return bool(torch is not None and torch.cuda.is_initialized())
    except Exception:
        return True


def evaluate_population(tokens, tok_offset, tok_len, consts, const_offset, const_count,
                        X, y, kind: int, mode: str = "o64", processes: Optional[int] = None,
                        subset=None, seed: int = 0, div_eps=None):
    """fitness float64[N] (or [len(subset)]) and status int8[...].

    ``subset`` restricts the evaluation to the listed program indices (in
    that order).  mode "bound" returns oracle.bound's first-order fitness
    bound per program instead (``div_eps``: the relative error bound of a
    division that is not correctly rounded, None for a correctly rounded one).
    """
    X = np.asarray(X, dtype=np.float32)
    y = np.asarray(y, dtype=np.float32)
    if subset is not None:
        idx = [int(p) for p in subset]
        tok_offset = np.asarray(tok_offset)[idx]
        tok_len = np.asarray(tok_len)[idx]
        const_offset = np.asarray(const_offset)[idx]
        const_count = np.asarray(const_count)[idx]
    N = len(tok_len)
    if processes and processes > 1 and _gpu_runtime_started():
        processes = None  # forking is unsafe once the GPU runtime runs threads
    if not processes or processes <= 1 or N < 2:
        _, f, s = _worker((tokens, consts, tok_offset, tok_len, const_offset, const_count,
                           X, y, kind, mode, 0, N, seed, div_eps))
        return f, s
    import multiprocessing as mp
    chunks = []
    step = max(1, math.ceil(N / (processes * 4)))
    for lo in range(0, N, step):
        chunks.append((tokens, consts, tok_offset, tok_len, const_offset, const_count,
                       X, y, kind, mode, lo, min(N, lo + step), seed, div_eps))
    f = np.empty(N)
    s = np.empty(N, dtype=np.int8)
    env_before = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        ctx = mp.get_context("fork")
        with ctx.Pool(processes) as pool:
            for lo, out, sts in pool.imap_unordered(_worker, chunks):
                f[lo:lo + len(out)] = out
                s[lo:lo + len(out)] = sts
    finally:
        if env_before is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = env_before
    return f, s
