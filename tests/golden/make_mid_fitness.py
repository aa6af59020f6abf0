"""Writes tests/golden/mid_fitness.txt: the oracle's values for every program
of the plain-mid workload (N=4096 postfix programs, lengths 5..64, D=5,
M=100000 cases, paper_2603_12292_amd.workloads.config_mid), for the MSE and
the correlation fitness 1 - r^2 (Eq. 1).

Only the oracle (oracle/) and the seeded input generator run here; the file
is test infrastructure for the GPU parity test that compares every program
of that workload (a GPU test process cannot run the oracle's process pool,
and the whole population takes minutes of CPU time).

Columns per line: program, kind (0 MSE, 1 CORR), status, F_O64, F_O32e,
F_O32p (seed 1), F_O32p (seed 2), B (oracle.bound's bound on the fitness
change of a binary32 evaluation with the library's operator accuracies,
gates.DIV_EPS for its division), floats written with repr (exact round trip).

    python tests/golden/make_mid_fitness.py [--processes P]
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import gates  # noqa: E402
import golden_mid  # noqa: E402
from oracle import population as opop  # noqa: E402
from paper_2603_12292_amd import workloads as wl  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--processes", type=int, default=len(os.sched_getaffinity(0)))
    a = ap.parse_args()
    w = wl.config_mid()
    ps = w.programs
    rows = {}
    for kind in (0, 1):
        t0 = time.time()
        cols = []
        for mode, seed in (("o64", 0), ("o32e", 0), ("o32p", 1), ("o32p", 2), ("bound", 0)):
            f, st = opop.evaluate_population(ps.tokens, ps.tok_offset, ps.tok_len, ps.consts, ps.const_offset,
                                             ps.const_count, w.data.X, w.data.y, kind, mode,
                                             processes=a.processes, seed=seed, div_eps=gates.DIV_EPS)
            cols.append(f)
            if mode == "o64":
                status = st
            print(f"kind {kind} {mode}{seed or ''}: {time.time() - t0:.0f} s", flush=True)
        rows[kind] = (status, cols)
    with open(golden_mid.PATH, "w") as out:
        out.write("# oracle values of every program of the plain-mid workload (workloads.config_mid)\n")
        out.write("# written by tests/golden/make_mid_fitness.py from oracle/ and the seeded generator alone\n")
        out.write(f"# inputs {golden_mid.input_hash(w)}\n")
        out.write("# program kind status F_O64 F_O32e F_O32p1 F_O32p2 bound\n")
        for kind in (0, 1):
            status, cols = rows[kind]
            for p in range(ps.n):
                out.write(f"{p} {kind} {int(status[p])} " + " ".join(repr(float(c[p])) for c in cols) + "\n")
    print(f"wrote {golden_mid.PATH}")


if __name__ == "__main__":
    main()
