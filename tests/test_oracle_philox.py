"""Pins of the oracle's Philox4x32-10 (CPU only)."""
import os

import numpy as np
import pytest

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(w, 16) for w in line.split()]
                rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_known_answer_vectors(ctr, key, out):
    assert list(philox.philox4x32_10(ctr, key)) == out
    got = philox.philox4x32_10_np(*[np.array([c]) for c in ctr], key[0], key[1])
    assert [int(g[0]) for g in got] == out


def test_vectorised_equals_scalar():
    rng = np.random.default_rng(1)
    c = rng.integers(0, 2**32, size=(4, 300), dtype=np.uint64)
    k = rng.integers(0, 2**32, size=2)
    vec = philox.philox4x32_10_np(c[0], c[1], c[2], c[3], k[0], k[1])
    for i in range(300):
        assert philox.philox4x32_10([int(v[i]) for v in c], k) == tuple(int(v[i]) for v in vec)


def test_below_and_unit_mappings():
    assert philox.below(0, 7) == 0 and philox.below(2**32 - 1, 7) == 6
    assert philox.unit(0) == 0.0 and philox.unit(2**32 - 1) == 1.0 - 2.0 ** -24
    assert philox.unit(0x12345678) == float(np.float32(philox.unit(0x12345678)))
    # chi-square uniformity of below(u, 7) over one million outputs
    w = philox.philox4x32_10_np(np.arange(250_000), 0, 0, 0, 123, 456)
    u = np.concatenate(w).astype(np.uint64)
    b = (u * np.uint64(7)) >> np.uint64(32)
    counts = np.bincount(b.astype(np.int64), minlength=7)
    e = len(u) / 7
    chi2 = float(np.sum((counts - e) ** 2 / e))
    assert chi2 < 22.46   # 6 dof, p = 0.001


def test_stream_layout():
    s = philox.Stream(seed=(7 << 32) | 9, index=3, generation=5, tag=2)
    blk1 = philox.philox4x32_10((3, 5, 1, 2), (9, 7))
    assert [s.draw(j) for j in range(4, 8)] == list(blk1)
