"""Constants of the library's binary32 sine, cosine (csrc/trig.h), exponential
and logarithm (csrc/beagle_device.h).

Run: python -m paper_2603_12292_amd.csrc.minimax  (prints the C++ constants)

1. Bits of 2/pi for the large-argument reduction (Payne and Hanek, "Radian
   reduction for trigonometric functions", SIGNUM Newsletter 18(1), 1983):
   pi comes from Machin's formula, pi/4 = 4 atan(1/5) - atan(1/239), in exact
   integer arithmetic with 320 guard bits, and floor(2^(224+1) / pi) gives
   bits 1..224 of 2/pi.
2. pi split into two binary64 numbers (Cody and Waite, "Software Manual for
   the Elementary Functions", 1980) for the reduction of |x| < 2^30, and 1/pi.
3. The polynomial on |r| <= pi/2 (with a 0.05 % margin): sin r = r + r^3
   S(r^2), S of degree 3, minimising the maximum relative error with
   Lawson's iteratively reweighted least squares (C. L. Lawson, 1961), then
   rounded to binary32.
4. log2(e) and ln(2) each split into a binary32 high part and the binary32
   nearest to the remainder (Cody and Waite), for the exponential and the
   logarithm built on the hardware base-2 functions.
"""
from __future__ import annotations

import functools

import numpy as np


def _atan_inv(n: int, one: int) -> int:
    """atan(1/n) * one, by its alternating series, in integers."""
    total, term, k, sign = 0, one // n, 1, 1
    while term:
        total += sign * (term // k)
        term //= n * n
        k += 2
        sign = -sign
    return total


def pi_fixed(bits: int) -> int:
    """floor-ish(pi * 2^bits) with `bits` correct bits (guard bits added)."""
    guard = 64
    one = 1 << (bits + guard)
    pi = 4 * (4 * _atan_inv(5, one) - _atan_inv(239, one))
    return pi >> guard


def two_over_pi_words(n_words: int = 7) -> list[int]:
    """32-bit words holding bits 1 .. 32*n_words of the fraction 2/pi."""
    nbits = 32 * n_words
    K = nbits + 320
    P = pi_fixed(K)                         # pi * 2^K
    frac = (1 << (nbits + 1 + K)) // P      # floor(2/pi * 2^nbits)
    return [(frac >> (32 * (n_words - 1 - i))) & 0xFFFFFFFF for i in range(n_words)]


def pi_split() -> tuple[float, float]:
    """(hi, lo): hi the binary64 nearest to pi, lo the binary64 nearest to pi - hi."""
    from fractions import Fraction
    P = pi_fixed(300)  # pi * 2^300
    hi = float(Fraction(P, 1 << 300))
    lo = float(Fraction(P, 1 << 300) - Fraction(hi))
    return hi, lo


def exp_log_splits() -> tuple[float, float, float, float]:
    """(log2e_hi, log2e_lo, ln2_hi, ln2_lo) as binary32 values (Python floats):
    hi the largest binary32 not above the constant, lo the binary32 nearest to
    the (positive) remainder, so that an infinite factor times hi and lo keeps
    one sign."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    ln2 = Decimal(2).ln()
    out = []
    for v in (1 / ln2, ln2):
        hi = np.float32(float(v))
        if Decimal(float(hi)) > v:
            hi = np.nextafter(hi, np.float32(0))
        lo = float(np.float32(float(v - Decimal(float(hi)))))
        out += [float(hi), lo]
    return tuple(out)


def _lawson(F, W, xs, deg, iters=400):
    A = np.stack([xs ** (2 * k) for k in range(deg)], 1)
    u = np.ones_like(xs) / len(xs)
    c = None
    for _ in range(iters):
        sw = np.sqrt(u) * W
        c, *_ = np.linalg.lstsq(A * sw[:, None], F * sw, rcond=None)
        e = np.abs(W * (F - A @ c))
        u = u * e
        u /= u.sum()
    return c


@functools.lru_cache(maxsize=None)
def poly_coefficients():
    xs = np.linspace(1e-5, np.pi / 2 * 1.0005, 50001)
    s = _lawson((np.sin(xs) - xs) / xs ** 3, xs ** 3 / np.sin(xs), xs, 4, iters=300)
    return tuple(np.float32(v) for v in s)


def main():
    words = two_over_pi_words()
    hi, lo = pi_split()
    s = poly_coefficients()
    print("two_over_pi bits 1..224:", ", ".join(f"0x{w:08X}u" for w in words))
    print(f"pi_hi = {hi.hex()}  pi_lo = {lo.hex()}  1/pi = {(1 / np.pi).hex()}")
    print("S =", ", ".join(f"{float(v).hex()}" for v in s))
    print("log2e hi, lo, ln2 hi, lo =", ", ".join(v.hex() for v in exp_log_splits()))


if __name__ == "__main__":
    main()
