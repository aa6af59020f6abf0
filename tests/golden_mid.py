"""Loader of tests/golden/mid_fitness.txt (see tests/golden/make_mid_fitness.py)."""
import hashlib
import os

import numpy as np

import gates

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mid_fitness.txt")


def input_hash(w) -> str:
    """sha256 of every input array of the workload: the golden values belong
    to exactly these programs and cases."""
    ps, d = w.programs, w.data
    h = hashlib.sha256()
    for a in (ps.tokens, ps.tok_offset, ps.tok_len, ps.consts, ps.const_offset, ps.const_count, d.X, d.y):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def load(w):
    """{kind: gates.Refs} for every program of workload w, after checking
    that the file was written for w's inputs."""
    rows = {0: [], 1: []}
    h = None
    with open(PATH) as f:
        for line in f:
            if line.startswith("# inputs "):
                h = line.split()[2]
            if line.startswith("#"):
                continue
            v = line.split()
            rows[int(v[1])].append([int(v[0]), int(v[2])] + [float(x) for x in v[3:]])
    assert h == input_hash(w), "golden values were written for other inputs: re-run make_mid_fitness.py"
    out = {}
    for kind, r in rows.items():
        a = np.array(r, dtype=np.float64)
        assert np.array_equal(a[:, 0], np.arange(w.programs.n))
        out[kind] = gates.Refs(a[:, 2], a[:, 1].astype(np.int8), a[:, 3], [a[:, 4], a[:, 5]], a[:, 6])
    return out
