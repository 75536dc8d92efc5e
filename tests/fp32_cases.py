"""Inputs and checks that pin FP32 accumulation (the mixed form's pass-1 product).

``order_free_case`` builds A (m x n) and an upper-triangular U (n x n) such
that one column of fl32(A) fl32(U) is a sum of three exact FP32 products
{1, 2^-24, 1.5 * 2^-50} (with signs).  Summed in FP32 -- in any order, by any
pairing, as one product per 4-term step of a matrix instruction or as one
fused multiply-add each -- the result is exactly 1, because every partial sum
that contains the leading 1 rounds back to 1 (2^-24 is half an ulp of 1 and
the tie goes to the even neighbour 1) and the two small terms sum to less than
half an ulp.  The exact sum 1 + 2^-24 + 1.5 * 2^-50 lies above that tie, so its
correctly rounded FP32 value is 1 + 2^-23: a product that accumulates in more
than FP32 precision and rounds once at the end gets that instead.  The three
terms sit at k = 0, 16 and 32, so on the GPU each one is a separate 4-term
matrix-instruction step.

``fp32_sum_stats`` compares an FP32 product with the exact product of the
FP32-rounded operands: the largest error relative to the standard FP32
summation bound n u32 (|A| |U|), and the fraction of entries that differ from
the correctly rounded exact value.  FP32 running sums round at almost every
step, so that fraction is large; a product accumulated in FP64 and rounded
once is correctly rounded almost everywhere.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np

U32 = 2.0 ** -24
TERMS = (1.0, 2.0 ** -24, 1.5 * 2.0 ** -50)
K_POS = (0, 16, 32)
DESIGNED_COL = 40


def order_free_case(m: int = 300, n: int = 48, seed: int = 0):
    """(A, U, rows, col): rows of A whose product with U's column ``col`` is an
    order-independent FP32 sum equal to +-1 (sign per row); every other entry
    of A U is a single exact product, except column ``col`` of the remaining
    random rows (a 4-term sum of random FP32 values)."""
    assert n > DESIGNED_COL
    rng = np.random.default_rng(seed)
    u = np.eye(n)
    for k in K_POS:
        u[k, DESIGNED_COL] = 1.0
    a = rng.standard_normal((m, n)).astype(np.float32).astype(np.float64)
    rows, signs = [], []
    for i, (perm, sign) in enumerate(itertools.product(itertools.permutations(TERMS), (1.0, -1.0))):
        r = 7 + 13 * i
        a[r, :] = rng.standard_normal(n).astype(np.float32)
        a[r, list(K_POS)] = [sign * t for t in perm]
        a[r, DESIGNED_COL] = 0.0
        rows.append(r)
        signs.append(sign)
    return a, u, np.array(rows), np.array(signs)


def exact_fp32_rounding_of_designed_sum(sign: float) -> float:
    """Correctly rounded FP32 value of sign * (1 + 2^-24 + 1.5 * 2^-50), exactly."""
    exact = sign * sum(Fraction(t) for t in TERMS)
    lo = np.float32(sign)
    hi = np.nextafter(lo, np.float32(2.0 * sign))
    dlo, dhi = abs(exact - Fraction(float(lo))), abs(exact - Fraction(float(hi)))
    assert dlo != dhi
    return float(lo if dlo < dhi else hi)


def all_fp32_orders_of_designed_sum(sign: float) -> set:
    """Every FP32 evaluation of the three designed terms: sequential sums in
    every order and every pairing (brute force over the parenthesizations)."""
    t = [np.float32(sign * x) for x in TERMS]
    out = set()
    for p in itertools.permutations(t):
        out.add(float(np.float32(np.float32(p[0] + p[1]) + p[2])))
        out.add(float(np.float32(p[0] + np.float32(p[1] + p[2]))))
    return out


def fp32_sum_stats(q32: np.ndarray, a: np.ndarray, u: np.ndarray):
    """(max error / FP32 bound, fraction not equal to the correctly rounded
    exact product) for q32 ~ fl32(a) fl32(u)."""
    a32 = np.asarray(a, np.float64).astype(np.float32).astype(np.float64)
    u32 = np.asarray(u, np.float64).astype(np.float32).astype(np.float64)
    n = a32.shape[1]
    exact = a32 @ u32           # error <= n 2^-53 |A||U|: negligible beside FP32
    bound = n * U32 * (np.abs(a32) @ np.abs(u32)) + 2.0 ** -149
    q = np.asarray(q32, np.float32).astype(np.float64)
    ratio = float(np.max(np.abs(q - exact) / bound))
    frac = float(np.mean(q != exact.astype(np.float32).astype(np.float64)))
    return ratio, frac
