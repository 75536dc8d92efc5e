"""Writes the exact worked examples under tests/golden/ (run: python tests/golden/make_golden.py).

The paper prints no numeric example, so these fixtures are constructed from the
definitions with exact rational arithmetic (``fractions.Fraction``), never from
the oracle or the GPU path:

* cholinv_exact_n*.json — Algorithm 2's postconditions A = L Lᵀ (L lower,
  positive diagonal) and Y = L^{-1}.  L is drawn with power-of-two diagonal and
  small integer off-diagonals, W = L Lᵀ is an integer matrix, and Y is the exact
  rational inverse.  Every entry is exactly representable in FP64, and (checked
  at generation time) so is every value Algorithm 2 forms on the way, so a
  correct FP64 CholInv reproduces L and Y bit for bit.
* qr_exact_*.json — reduced QR (Section "QR Factorization": Q with orthonormal
  columns, R upper triangular, here with positive diagonal, which makes it
  unique for full-rank A) of matrices with exact rational Q and R.
"""
from __future__ import annotations

import json
import os
import random
from fractions import Fraction as F

HERE = os.path.dirname(os.path.abspath(__file__))


def exact_lower_inverse(l):
    n = len(l)
    y = [[F(0)] * n for _ in range(n)]
    for j in range(n):
        for i in range(j, n):
            s = F(1) if i == j else F(0)
            for k in range(j, i):
                s -= l[i][k] * y[k][j]
            y[i][j] = s / l[i][i]
    return y


def as_float_exact(x: F) -> float:
    f = float(x)
    if F(f) != x:
        raise ValueError(f"{x} is not exactly representable")
    return f


def cholinv_example(n: int, seed: int):
    rnd = random.Random(seed)
    l = [[F(0)] * n for _ in range(n)]
    for i in range(n):
        l[i][i] = F(2 ** rnd.randint(0, 2))
        for j in range(i):
            l[i][j] = F(rnd.randint(-3, 3))
    w = [[sum(l[i][k] * l[j][k] for k in range(n)) for j in range(n)] for i in range(n)]
    y = exact_lower_inverse(l)
    return {
        "cite": "Algorithm 2 (CholInv) postconditions: A = L L^T, L lower, Y = L^-1",
        "construction": f"L: diag 2^U{{0,1,2}}, strict lower U{{-3..3}} from random.Random({seed}); "
                        "W = L L^T; Y = exact rational inverse",
        "n": n,
        "W": [[as_float_exact(x) for x in row] for row in w],
        "L": [[as_float_exact(x) for x in row] for row in l],
        "Y": [[as_float_exact(x) for x in row] for row in y],
    }


def qr_examples():
    # [[3,1],[4,2]]: a = (3,4), |a| = 5, R12 = a.b/|a| = 11/5, b - (11/25) a = (-8/25, 6/25),
    # |.| = 2/5; Q = [[3/5,-4/5],[4/5,3/5]].
    ex2 = {
        "cite": "reduced QR definition (Section QR Factorization); n = 2 closed form "
                "R11 = |a|, R12 = a.b/|a|, R22 = |b - (a.b/|a|^2) a|",
        "A": [[3.0, 1.0], [4.0, 2.0]],
        "Q": [["3/5", "-4/5"], ["4/5", "3/5"]],
        "R": [["5", "11/5"], ["0", "2/5"]],
    }
    # 4x3 with orthogonal integer columns scaled: A = Q R with Q = H/2 (H Hadamard-like
    # 4x3 columns of +-1) and R integer upper triangular with positive diagonal.
    h = [[1, 1, 1], [1, -1, 1], [1, 1, -1], [1, -1, -1]]
    q = [[F(h[i][j], 2) for j in range(3)] for i in range(4)]
    r = [[F(2), F(1), F(-3)], [F(0), F(4), F(2)], [F(0), F(0), F(1)]]
    a = [[sum(q[i][k] * r[k][j] for k in range(3)) for j in range(3)] for i in range(4)]
    ex3 = {
        "cite": "reduced QR definition (Section QR Factorization); unique for full rank with diag(R) > 0",
        "A": [[as_float_exact(x) for x in row] for row in a],
        "Q": [[str(x) for x in row] for row in q],
        "R": [[str(x) for x in row] for row in r],
    }
    return {"qr_exact_2x2.json": ex2, "qr_exact_4x3.json": ex3}


def main():
    for n, seed in ((2, 0), (3, 1), (5, 2), (8, 3), (13, 4), (16, 5), (33, 6)):
        ex = cholinv_example(n, seed)
        with open(os.path.join(HERE, f"cholinv_exact_n{n}.json"), "w") as f:
            json.dump(ex, f, indent=1)
    for name, ex in qr_examples().items():
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(ex, f, indent=1)


if __name__ == "__main__":
    main()
