"""Plain CPU FP64 CholeskyQR2 — the oracle the HIP path is checked against.

Test infrastructure: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.  Written from the paper (Hutter & Solomonik,
"Communication-avoiding CholeskyQR2 for rectangular matrices"):

* sequential routines and their costs: Section "Preliminaries"
  (Syrk = AᵀA costs m n^2, MM = AB costs 2 m n k);
* recursive Cholesky, recursive triangular inverse and their combination
  CholInv: Section "Cholesky Factorization", Algorithm 2;
* CholeskyQR (CQR): Algorithm 4; CholeskyQR2 (CQR2): Algorithm 5.

Everything is IEEE FP64 with numpy's library GEMM as the only primitive; no
blocking, fusion or reordering beyond the recursive halving that Algorithm 2
itself prescribes.  Readings where the paper is silent:

* Syrk produces the lower triangle; the upper is never read (Alg. 2 reads A11,
  A21, A22 only).  Here the full symmetric W is returned for convenience.
* Odd n is split at h = floor(n/2) (the paper writes n/2).
* The recursion goes down to n = 1 exactly as Algorithm 2's base case.
* A non-positive or NaN pivot (the paper assumes SPD input) raises
  ``NotSPD(j)`` with the 1-based column j, following LAPACK potrf's info.
* Q is formed by multiplying by the explicit inverse R^{-1} (Algorithm 4's MM),
  not by a triangular solve.
* The second pass factors the stored Q1 (in the mixed form: the FP32 values,
  converted exactly to FP64).

Mixed precision (``mm_fp32``, ``cqr2_mixed``): the paper fixes no reduced
precision.  The reading taken is the one the GPU path offers: pass 1's
Q1 = A R1^{-1} with both operands rounded to FP32 and every product and
running sum kept in FP32 (the library's single-precision GEMM), everything
else FP64.  Its FP32 accumulation is pinned by a designed input whose FP32
sum is the same in every order yet differs from the correctly rounded exact
sum, by the standard FP32 summation error bound, and by the fraction of
entries that differ from the correctly rounded product (an FP64-accumulating
mistake makes that fraction vanish).

Shifted CholeskyQR3 (``scqr3``): the paper names the shifted variant of
Fukaya et al. (its Conclusion and the CholeskyQR2 background of its
Introduction) as an unconditionally stable extension that needs only minimal
changes, without defining it.  It is written here from that published method:
one CholeskyQR of A with W + s I in place of W, s = 11 (m n + n (n + 1)) u
||A||_F^2 (u = 2^-53, ||A||_F^2 = trace W), followed by CholeskyQR2 of the
result; R = R3 R2 R1.  Parity of this form is pinned to Householder QR, closed
forms and exact scaling, not to anything the paper prints.

Partial inverse (``cholinv_partial``, ``cqr2_partial``): the alternative the
paper describes for its 3D-CQR2 (Section "Communication-avoiding
CholeskyQR2"): only triangular diagonal blocks of dimension n_o are inverted
and Q is found by several matrix multiplications instead of one with the full
R^{-1}; its experiments tune the recursion level down to which the inverse
is formed (InverseDepth).  Reading taken: with depth d, the top d levels of
Algorithm 2's recursion do not form Y21 (the inverse stays block diagonal
with the blocks of level d), and every product that needs the inverse of such
a block -- L21 = A21 L11^{-T} inside the recursion and Q = A R^{-1} -- is
formed by block substitution over the inverted diagonal blocks, one matrix
multiplication pair per block.  d = 0 is Algorithm 2 itself.
"""
from __future__ import annotations

import math

import numpy as np


class NotSPD(ArithmeticError):
    """Cholesky breakdown: pivot at 1-based column ``j`` is <= 0 or NaN."""

    def __init__(self, j: int):
        super().__init__(f"matrix is not numerically SPD (pivot {j})")
        self.j = j


def syrk(a: np.ndarray) -> np.ndarray:
    """W = AᵀA (Preliminaries, Syrk).  Returns the symmetric n x n W in FP64.

    The lower triangle is the product itself; the upper triangle is mirrored
    from it so no consumer can depend on it.
    """
    a = np.asarray(a, dtype=np.float64)
    w = a.T @ a
    low = np.tril(w)
    return low + np.tril(w, -1).T


def cholinv(a: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """[L, Y] = CholInv(A) (Algorithm 2): A = L Lᵀ with L lower, Y = L^{-1}.

    The recursion halves A.  The leading diagonal block gives its own factor
    and inverse; the off-diagonal block of L is the leading inverse applied
    to A's off-diagonal block; the trailing block's factor and inverse come
    from its Schur complement; and the off-diagonal block of the inverse is
    minus the trailing inverse times L's off-diagonal block times the leading
    inverse (multiplied right to left, as Algorithm 3 orders it).  A 1 x 1
    block is its square root and that root's reciprocal.  Only the lower
    triangle of ``a`` is read.
    """
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("CholInv needs a square matrix")
    if n == 0:
        return np.zeros((0, 0)), np.zeros((0, 0))
    if n == 1:
        piv = a[0, 0]
        if not piv > 0.0:          # catches <= 0 and NaN
            raise NotSPD(1)
        l = math.sqrt(piv)
        return np.array([[l]]), np.array([[1.0 / l]])
    h = n // 2
    l11, y11 = cholinv(a[:h, :h])
    l21 = a[h:, :h] @ y11.T
    schur = a[h:, h:] - l21 @ l21.T
    try:
        l22, y22 = cholinv(schur)
    except NotSPD as e:
        raise NotSPD(e.j + h) from None
    u = l21 @ y11
    y21 = -(y22 @ u)
    l = np.zeros((n, n))
    y = np.zeros((n, n))
    l[:h, :h] = l11
    l[h:, :h] = l21
    l[h:, h:] = l22
    y[:h, :h] = y11
    y[h:, :h] = y21
    y[h:, h:] = y22
    return l, y


def cqr(a: np.ndarray):
    """[Q, R] = CQR(A) (Algorithm 4).

    W = Syrk(A); Rᵀ, R^{-T} = CholInv(W); Q = MM(A, R^{-1}).
    Returns (Q, R, R^{-1}).
    """
    a = np.asarray(a, dtype=np.float64)
    w = syrk(a)
    l, y = cholinv(w)
    r = l.T.copy()
    rinv = y.T.copy()
    q = a @ rinv
    return q, r, rinv


def upper_product(r2: np.ndarray, r1: np.ndarray) -> np.ndarray:
    """R = MM(R2, R1) for two upper-triangular factors (Algorithm 5, last line)."""
    return np.asarray(r2, dtype=np.float64) @ np.asarray(r1, dtype=np.float64)


def cqr2(a: np.ndarray, return_intermediates: bool = False):
    """[Q, R] = CQR2(A) (Algorithm 5): two CQR passes, then R = R2 R1.

    With ``return_intermediates`` also returns a dict with W1, R1, R1^{-1},
    Q1, W2, R2, R2^{-1}.  A breakdown in the second pass is reported as
    ``NotSPD(n + j)``.
    """
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[1]
    q1, r1, r1inv = cqr(a)
    try:
        q, r2, r2inv = cqr(q1)
    except NotSPD as e:
        raise NotSPD(n + e.j) from None
    r = upper_product(r2, r1)
    if not return_intermediates:
        return q, r
    return q, r, {
        "W1": syrk(a), "R1": r1, "R1inv": r1inv, "Q1": q1,
        "W2": syrk(q1), "R2": r2, "R2inv": r2inv,
    }


def mm_fp32(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """C = MM(fl32(A), fl32(B)) in FP32 arithmetic, returned as FP32.

    Both operands are rounded to FP32 (round to nearest even); the library's
    single-precision GEMM then forms every product and every running sum in
    FP32, in its own summation order.
    """
    a32 = np.asarray(a, dtype=np.float64).astype(np.float32)
    b32 = np.asarray(b, dtype=np.float64).astype(np.float32)
    return a32 @ b32


def cqr2_mixed(a: np.ndarray, return_intermediates: bool = False):
    """CQR2 with pass 1's Q1 = A R1^{-1} formed in FP32 (``mm_fp32``).

    Gram, CholInv and everything in pass 2 stay FP64; pass 2 factors the stored
    FP32 Q1 after exact conversion to FP64.  Not in the paper (it fixes no
    precision); it is the reduced-precision variant the GPU path offers.
    """
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[1]
    w1 = syrk(a)
    l1, y1 = cholinv(w1)
    r1 = l1.T.copy()
    r1inv = y1.T.copy()
    q1_32 = mm_fp32(a, r1inv)
    q1 = q1_32.astype(np.float64)
    try:
        q, r2, r2inv = cqr(q1)
    except NotSPD as e:
        raise NotSPD(n + e.j) from None
    r = upper_product(r2, r1)
    if not return_intermediates:
        return q, r
    return q, r, {"W1": w1, "R1": r1, "R1inv": r1inv, "Q1": q1,
                  "R2": r2, "R2inv": r2inv}


UNIT_ROUNDOFF = 2.0 ** -53


def cholesky_shift(w: np.ndarray, m: int) -> float:
    """Shift s = 11 (m n + n (n + 1)) u trace(W) of shifted CholeskyQR (trace W = ||A||_F^2)."""
    n = w.shape[0]
    return 11.0 * (m * n + n * (n + 1)) * UNIT_ROUNDOFF * float(np.trace(w))


def scqr3(a: np.ndarray, return_intermediates: bool = False):
    """[Q, R] = shifted CholeskyQR3: CQR with a shifted Gram, then CQR2.

    Breakdowns report the column of the pass: j, n + j or 2 n + j.
    """
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    w = syrk(a)
    s = cholesky_shift(w, m)
    l1, y1 = cholinv(w + s * np.eye(n))
    r1 = l1.T.copy()
    q1 = a @ y1.T
    try:
        q2, r2, _ = cqr(q1)
    except NotSPD as e:
        raise NotSPD(n + e.j) from None
    try:
        q, r3, _ = cqr(q2)
    except NotSPD as e:
        raise NotSPD(2 * n + e.j) from None
    r = upper_product(r3, upper_product(r2, r1))
    if not return_intermediates:
        return q, r
    return q, r, {"shift": s, "R1": r1, "Q1": q1, "R2": r2, "R3": r3}


def lstsq(a: np.ndarray, b: np.ndarray):
    """Least-squares solution x = argmin ||A x - b|| from CholeskyQR2.

    One of the uses the paper's Introduction names for the QR factorization
    (least-squares problems): with
    A = Q R, x = R^{-1} (Qᵀ b).  R^{-1} is applied as the method forms it,
    through the explicit triangular inverses of the two passes,
    R^{-1} = (R2 R1)^{-1} = R1^{-1} R2^{-1}.  b: m x k.
    Returns (x, Q, R).
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    q, r, it = cqr2(a, return_intermediates=True)
    c = q.T @ b
    x = it["R1inv"] @ (it["R2inv"] @ c)
    return x, q, r


def solve_right_lt(b: np.ndarray, l: np.ndarray, y: np.ndarray, blocks) -> np.ndarray:
    """X = B L^{-T} by block substitution (X Lᵀ = B, L lower triangular).

    ``y`` holds the inverses of L's diagonal blocks ``blocks`` (a list of
    (start, stop) column ranges covering 0..n in order); nothing else of y is
    read.  Block j: X_j = (B_j - X_{<j} L_{j,<j}ᵀ) Y_jjᵀ.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    for c0, c1 in blocks:
        t = b[:, c0:c1] - x[:, :c0] @ l[c0:c1, :c0].T
        x[:, c0:c1] = t @ y[c0:c1, c0:c1].T
    return x


def cholinv_partial(a: np.ndarray, depth: int):
    """[L, Y, blocks] = CholInv with the inverse formed only below ``depth``.

    At a level with depth > 0: L11, Y11 = CholInv_partial(A11, depth - 1);
    L21 = A21 L11^{-T} by block substitution over Y11's diagonal blocks;
    L22, Y22 = CholInv_partial(A22 - L21 L21ᵀ, depth - 1); Y21 is not formed
    (zero).  depth == 0 (or n == 1) is Algorithm 2 (``cholinv``).  ``blocks``
    lists the diagonal blocks of Y that are inverses of L's.
    """
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    if depth <= 0 or n <= 1:
        l, y = cholinv(a)
        return l, y, [(0, n)]
    h = n // 2
    l11, y11, b11 = cholinv_partial(a[:h, :h], depth - 1)
    l21 = solve_right_lt(a[h:, :h], l11, y11, b11)
    schur = a[h:, h:] - l21 @ l21.T
    try:
        l22, y22, b22 = cholinv_partial(schur, depth - 1)
    except NotSPD as e:
        raise NotSPD(e.j + h) from None
    l = np.zeros((n, n))
    y = np.zeros((n, n))
    l[:h, :h] = l11
    l[h:, :h] = l21
    l[h:, h:] = l22
    y[:h, :h] = y11
    y[h:, h:] = y22
    return l, y, b11 + [(h + c0, h + c1) for c0, c1 in b22]


def cqr_partial(a: np.ndarray, depth: int):
    """CQR (Algorithm 4) with the partial inverse: W = Syrk(A);
    L, Y, blocks = CholInv_partial(W, depth); R = Lᵀ; Q = A R^{-1} = A L^{-T}
    by block substitution.  Returns (Q, R, Y, blocks)."""
    a = np.asarray(a, dtype=np.float64)
    w = syrk(a)
    l, y, blocks = cholinv_partial(w, depth)
    q = solve_right_lt(a, l, y, blocks)
    return q, l.T.copy(), y, blocks


def cqr2_partial(a: np.ndarray, depth: int):
    """CQR2 (Algorithm 5) on ``cqr_partial``: returns (Q, R)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[1]
    q1, r1, _, _ = cqr_partial(a, depth)
    try:
        q, r2, _, _ = cqr_partial(q1, depth)
    except NotSPD as e:
        raise NotSPD(n + e.j) from None
    return q, upper_product(r2, r1)
