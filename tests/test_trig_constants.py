"""The constants of the device sine/cosine (csrc/trig.h), exponential and
logarithm (csrc/beagle_device.h) are the ones csrc/minimax.py derives, and
that derivation is pinned independently."""
import math
import os
import re
from decimal import Decimal, getcontext

import numpy as np

from paper_2603_12292_amd.csrc import minimax

HDR = os.path.join(os.path.dirname(minimax.__file__), "trig.h")


def _pi_gauss_legendre(digits=100):
    getcontext().prec = digits
    a, b, t, p = Decimal(1), Decimal(1) / Decimal(2).sqrt(), Decimal(1) / 4, Decimal(1)
    for _ in range(9):
        an = (a + b) / 2
        b = (a * b).sqrt()
        t -= p * (a - an) ** 2
        a = an
        p *= 2
    return (a + b) ** 2 / (4 * t)


def test_two_over_pi_bits_against_gauss_legendre():
    words = minimax.two_over_pi_words()
    v = int("".join(f"{w:032b}" for w in words), 2)
    ref = int((Decimal(2) / _pi_gauss_legendre()) * (Decimal(2) ** 224))
    assert v == ref
    assert abs(v / 2.0 ** 224 - 2 / math.pi) < 1e-16


def test_pi_split():
    hi, lo = minimax.pi_split()
    assert hi == math.pi
    pi = _pi_gauss_legendre()
    assert abs((Decimal(hi) + Decimal(lo)) - pi) < Decimal(2) ** -105
    assert abs(lo) < 2.0 ** -52


def test_polynomial_accuracy():
    s = minimax.poly_coefficients()
    r = np.linspace(1e-6, np.pi / 2, 200001)
    p = np.polyval([float(c) for c in s[::-1]], r * r)
    rel = np.abs((r + r ** 3 * p) / np.sin(r) - 1)
    assert rel.max() < 0.3 * 2.0 ** -24


def test_header_holds_the_derived_constants():
    with open(HDR) as f:
        text = f.read()
    words = minimax.two_over_pi_words()
    table = re.search(r"two_over_pi\[7\] = \{([^}]*)\}", text).group(1)
    assert [int(w.strip().rstrip("u"), 16) for w in table.split(",")] == words
    hi, lo = minimax.pi_split()
    assert hi.hex() in text and lo.hex() in text and (1 / math.pi).hex() in text
    # pi/2 for the cosine of the shared reduction: the exact halves
    assert (hi / 2).hex() in text and (lo / 2).hex() in text
    body = text[text.index("float sin_poly"):text.index("trig_reduce_small")]
    lits = [float.fromhex(x.rstrip("f")) for x in re.findall(r"-?0x1\.[0-9a-f]+p[-+]?\d+f", body)]
    assert sorted(lits) == sorted(float(c) for c in minimax.poly_coefficients())


def _c_hex(v: float) -> str:
    """binary32 value as the kernels spell it: 0x1.hhhhhhp+e (6 hex digits)."""
    m, e = v.hex().split("p")
    sign = "-" if m.startswith("-") else ""
    m = m.lstrip("-")
    return f"{sign}{m[:10].ljust(10, '0')}p{e}"


def test_exp_log_splits():
    l2e_hi, l2e_lo, ln2_hi, ln2_lo = minimax.exp_log_splits()
    for hi, lo, exact in ((l2e_hi, l2e_lo, 1 / math.log(2)), (ln2_hi, ln2_lo, math.log(2))):
        assert np.float32(hi) == hi and np.float32(lo) == lo
        # lo is the binary32 nearest to the positive remainder
        assert abs(hi + lo - exact) <= float(np.spacing(np.float32(lo))) / 2 and lo > 0
        assert abs(lo) <= np.spacing(np.float32(hi))
    with open(os.path.join(os.path.dirname(minimax.__file__), "beagle_device.h")) as f:
        text = f.read()
    for v in minimax.exp_log_splits():
        assert _c_hex(v) in text, _c_hex(v)
