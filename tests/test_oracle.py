"""Pins for the CPU oracle: each checks it against something other than itself.

* exact worked examples (tests/golden, exact rational arithmetic) — CholInv
  reproduces L and Y bit for bit, for even and odd n;
* brute force — integer Gram matrices computed exactly with Python ints;
* library routines for special cases — LAPACK potrf/trtri (scipy) for
  CholInv, LAPACK Householder QR for CQR2's R (Introduction: CQR2 is as
  accurate as Householder QR for cond(A) = O(eps^{-1/2}));
* closed forms — n = 1 and n = 2 QR, exact 4x3 QR;
* 50-digit Gram-Schmidt (mpmath) on tiny inputs;
* invariants — A = QR, QᵀQ = I, R upper with positive diagonal, power-of-two
  scaling is exact;
* FP32 accumulation of the mixed form — a designed sum whose FP32 value is
  the same in every order but is not the correctly rounded exact sum, the FP32
  summation error bound, and the share of entries that differ from the
  correctly rounded product;
* planted mistakes — mutated copies of the oracle must fail the pins above.
"""
import json
import math
import os
from fractions import Fraction as F

import numpy as np
import pytest
import scipy.linalg

import oracle
from tests import fp32_cases
from oracle import cqr2_ref
from synth import gdv_matrix, integer_matrix

GOLD = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _frac_matrix(rows):
    return np.array([[float(F(x)) for x in r] for r in rows])


# ---------------------------------------------------------------- Syrk ---

@pytest.mark.parametrize("m,n,seed", [(1, 1, 0), (7, 3, 1), (64, 16, 2), (1000, 33, 3)])
def test_syrk_exact_integer_gram(m, n, seed):
    a = integer_matrix(m, n, 64, seed)
    w = oracle.syrk(a)
    ai = a.astype(np.int64)
    exact = [[int(sum(int(ai[k, i]) * int(ai[k, j]) for k in range(m))) for j in range(n)]
             for i in range(n)]
    assert np.array_equal(w, np.array(exact, dtype=np.float64))


def test_syrk_shape_and_symmetry():
    a = gdv_matrix(50, 7, 10.0, 9)
    w = oracle.syrk(a)
    assert w.shape == (7, 7)
    assert np.array_equal(w, w.T)


# ------------------------------------------------------------- CholInv ---

@pytest.mark.parametrize("n", [2, 3, 5, 8, 13, 16, 33])
def test_cholinv_exact_examples(n):
    d = _gold(f"cholinv_exact_n{n}.json")
    l, y = oracle.cholinv(np.array(d["W"]))
    assert np.array_equal(l, np.array(d["L"]))
    assert np.array_equal(y, np.array(d["Y"]))


def test_cholinv_reads_lower_triangle_only():
    d = _gold("cholinv_exact_n8.json")
    w = np.array(d["W"])
    w_polluted = np.tril(w) + np.triu(np.full_like(w, 1e300), 1)
    l, y = oracle.cholinv(w_polluted)
    assert np.array_equal(l, np.array(d["L"]))
    assert np.array_equal(y, np.array(d["Y"]))


@pytest.mark.parametrize("n,kappa", [(1, 1.0), (4, 10.0), (31, 1e3), (64, 1e4), (128, 1e6)])
def test_cholinv_matches_lapack(n, kappa):
    a = gdv_matrix(max(2 * n, 8), n, math.sqrt(kappa), 100 + n)
    w = oracle.syrk(a)
    l, y = oracle.cholinv(w)
    l_ref = scipy.linalg.cholesky(w, lower=True)
    y_ref, info = scipy.linalg.lapack.dtrtri(l_ref, lower=1)
    assert info == 0
    cw = np.linalg.cond(w)
    tol = 20 * n * U * cw
    assert oracle.rel_fro(l, l_ref) <= tol
    assert oracle.rel_fro(y, np.tril(y_ref)) <= tol
    # invariants of Algorithm 2's postcondition
    assert np.array_equal(l, np.tril(l)) and np.array_equal(y, np.tril(y))
    assert np.all(np.diag(l) > 0)
    assert np.linalg.norm(l @ l.T - w) <= 10 * n * U * np.linalg.norm(w)
    assert np.linalg.norm(y @ l - np.eye(n)) <= 10 * n * U * cw ** 0.5 * 10


@pytest.mark.parametrize("n", [130, 200, 256])
def test_cholinv_split_at_128_matches_oracle(n):
    """The GPU's one-workgroup CholInv for 128 < n <= 256 (and the recursion
    above 128) splits W at h = 128, not at floor(n/2): R11 and R11^-1 from
    CholInv(W11), R12 = R11^-T W12, the Schur complement S = W22 - R12^T R12,
    R22 and R22^-1 from CholInv(S), and (R^-1)12 = -R11^-1 R12 R22^-1.  In
    exact arithmetic that is the same factor and inverse as Algorithm 2's
    halving (the Cholesky factor is unique); here the block equations, written
    with the oracle's CholInv on the diagonal blocks, agree with the oracle to
    rounding, and a sign slip in the coupling block is caught."""
    a = gdv_matrix(3 * n, n, 1e3, 300 + n)
    w = oracle.syrk(a)
    l, y = oracle.cholinv(w)
    h = 128
    l11, y11 = oracle.cholinv(w[:h, :h])
    r11, ri11 = l11.T, y11.T
    r12 = ri11.T @ w[:h, h:]
    s = w[h:, h:] - r12.T @ r12
    l22, y22 = oracle.cholinv(s)
    r22, ri22 = l22.T, y22.T
    ri12 = -(ri11 @ r12) @ ri22
    r = np.block([[r11, r12], [np.zeros((n - h, h)), r22]])
    ri = np.block([[ri11, ri12], [np.zeros((n - h, h)), ri22]])
    tol = 50 * n * U * np.linalg.cond(w)
    assert oracle.rel_fro(r, l.T) <= tol
    assert oracle.rel_fro(ri, y.T) <= tol
    assert np.linalg.norm(ri @ r - np.eye(n)) <= tol * n
    wrong = np.block([[ri11, -ri12], [np.zeros((n - h, h)), ri22]])
    assert oracle.rel_fro(wrong, y.T) > 1e-3


def _blocked_cholinv(w, b=128, drop_prev_diag=False):
    """Algorithm 2 with the split at the first b columns at every level,
    unrolled into a loop over b-column blocks in the order the GPU runs it for
    n >= 512: base(k) on the diagonal block, the inverse's block column k from
    the leading inverse, panel(k) = R_kk^-T W_{>k,k}^T, and update(k) in three
    parts -- the next block column below its diagonal block, the trailing lower
    triangle below block row k + 2, and the diagonal block k + 1 taking
    update(k - 1) and update(k) together.  Only the lower triangle of the
    working copy is read or updated."""
    n = w.shape[0]
    lw = np.tril(w).copy()
    r = np.zeros((n, n))
    ri = np.zeros((n, n))
    nb = (n + b - 1) // b
    c = [min(k * b, n) for k in range(nb + 3)]

    def sub_lower(r0, c0, upd):
        rows = np.arange(r0, r0 + upd.shape[0])[:, None]
        cols = np.arange(c0, c0 + upd.shape[1])[None, :]
        lw[r0:r0 + upd.shape[0], c0:c0 + upd.shape[1]] -= np.where(rows >= cols, upd, 0.0)

    for k in range(nb):
        c0, c1 = c[k], c[k + 1]
        blk = np.tril(lw[c0:c1, c0:c1])
        lkk, ykk = oracle.cholinv(blk + np.tril(blk, -1).T)
        r[c0:c1, c0:c1], ri[c0:c1, c0:c1] = lkk.T, ykk.T
        if k >= 1:
            x = r[:c0, c0:c1] @ ri[c0:c1, c0:c1]
            ri[:c0, c0:c1] = -(ri[:c0, :c0] @ x)
        if c1 >= n:
            break
        c2, c3 = c[k + 2], c[k + 3]
        r[c0:c1, c1:] = ri[c0:c1, c0:c1].T @ lw[c1:, c0:c1].T
        sub_lower(c2, c1, r[c0:c1, c2:].T @ r[c0:c1, c1:c2])
        if c3 < n:
            sub_lower(c3, c2, r[c0:c1, c3:].T @ r[c0:c1, c2:])
        kr = b if (k == 0 or drop_prev_diag) else 2 * b
        rd = r[c1 - kr:c1, c1:c2]
        sub_lower(c1, c1, rd.T @ rd)
    return r, ri


@pytest.mark.parametrize("n", [520, 640])
def test_cholinv_blocked_lookahead_form_matches_oracle(n):
    """The GPU's CholInv for n >= 512 is Algorithm 2 split at 128 columns at
    every level, run block by block with look-ahead.  Written out with the
    oracle's CholInv on the diagonal blocks, that schedule of block updates
    reproduces the oracle's factor and inverse to rounding (every block of W
    takes each step's update exactly once), and dropping update(k - 1) from the
    diagonal block's combined update is caught."""
    a = gdv_matrix(3 * n, n, 1e3, 500 + n)
    w = oracle.syrk(a)
    l, y = oracle.cholinv(w)
    r, ri = _blocked_cholinv(w)
    tol = 50 * n * U * np.linalg.cond(w)
    assert oracle.rel_fro(r, l.T) <= tol
    assert oracle.rel_fro(ri, y.T) <= tol
    assert np.array_equal(r, np.triu(r)) and np.array_equal(ri, np.triu(ri))
    try:
        rb, _ = _blocked_cholinv(w, drop_prev_diag=True)
        assert oracle.rel_fro(rb, l.T) > 1e-3
    except oracle.NotSPD:
        pass  # the mutant may also break down on a later block


def test_cholinv_breakdown_columns():
    d = _gold("cholinv_exact_n8.json")
    w = np.array(d["W"])
    for j in (0, 3, 7):
        wz = w.copy()
        wz[j, :] = 0.0
        wz[:, j] = 0.0
        with pytest.raises(oracle.NotSPD) as e:
            oracle.cholinv(wz)
        assert e.value.j == j + 1
    wn = w.copy()
    wn[5, 5] = np.nan
    with pytest.raises(oracle.NotSPD) as e:
        oracle.cholinv(wn)
    assert e.value.j == 6
    with pytest.raises(oracle.NotSPD) as e:
        oracle.cholinv(-np.eye(3))
    assert e.value.j == 1


# ---------------------------------------------------------------- CQR2 ---

def test_qr_closed_form_n1():
    a = np.array([[1.0], [2.0], [2.0]])
    q, r = oracle.cqr2(a)
    assert abs(r[0, 0] - 3.0) <= 4 * U * 3.0
    assert np.max(np.abs(q[:, 0] - a[:, 0] / 3.0)) <= 4 * U
    rng = np.random.default_rng(3)
    for _ in range(20):
        v = rng.standard_normal((int(rng.integers(1, 200)), 1))
        q, r = oracle.cqr2(v)
        nrm = np.linalg.norm(v)
        assert abs(r[0, 0] - nrm) <= 8 * U * nrm
        assert np.max(np.abs(q - v / nrm)) <= 8 * U


@pytest.mark.parametrize("name", ["qr_exact_2x2.json", "qr_exact_4x3.json"])
def test_qr_exact_closed_form(name):
    d = _gold(name)
    a = np.array(d["A"])
    q, r = oracle.cqr2(a)
    q_ref, r_ref = _frac_matrix(d["Q"]), _frac_matrix(d["R"])
    assert np.max(np.abs(q - q_ref)) <= 16 * U
    assert np.max(np.abs(r - r_ref)) <= 16 * U * np.abs(r_ref).max()
    assert np.array_equal(r, np.triu(r))


def test_qr_n2_closed_form_random():
    rng = np.random.default_rng(11)
    for _ in range(20):
        m = int(rng.integers(2, 50))
        a, b = rng.standard_normal(m), rng.standard_normal(m)
        q, r = oracle.cqr2(np.stack([a, b], axis=1))
        na = np.linalg.norm(a)
        r12 = a @ b / na
        r22 = np.linalg.norm(b - (a @ b / na ** 2) * a)
        ref = np.array([[na, r12], [0.0, r22]])
        assert np.max(np.abs(r - ref)) <= 64 * U * np.abs(ref).max() * max(1.0, na / r22)


@pytest.mark.parametrize("m,n,kappa,seed", [
    (4096, 64, 1e3, 1), (2000, 128, 1e6, 2), (3000, 256, 1e6, 4), (500, 17, 1e4, 5),
    (64, 64, 1e2, 6)])
def test_cqr2_matches_householder(m, n, kappa, seed):
    a = gdv_matrix(m, n, kappa, seed)
    q, r = oracle.cqr2(a)
    qh, rh = oracle.householder_qr_posdiag(a)
    assert oracle.orthogonality(q) <= 1e-12
    assert oracle.residual(a, q, r) <= 1e-13
    assert oracle.rel_fro(r, rh) <= 1e-9
    assert oracle.rel_fro(q, qh) <= 1e-9
    assert np.array_equal(r, np.triu(r)) and np.all(np.diag(r) > 0)


def test_cqr2_refinement_factor_near_identity():
    # Introduction: the second CholeskyQR's triangular factor is near the identity.
    a = gdv_matrix(3000, 40, 1e5, 8)
    _, _, it = oracle.cqr2(a, return_intermediates=True)
    assert np.linalg.norm(it["R2"] - np.eye(40)) <= 1e-4
    assert np.linalg.norm(it["R2"] - np.eye(40)) > 0.0


def test_cqr2_power_of_two_scaling_is_exact():
    a = gdv_matrix(300, 12, 1e4, 12)
    q, r = oracle.cqr2(a)
    for k in (-7, 3, 20):
        qs, rs = oracle.cqr2(a * 2.0 ** k)
        assert np.array_equal(qs, q)
        assert np.array_equal(rs, r * 2.0 ** k)


def test_cqr2_mpmath_gram_schmidt():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    rng = np.random.default_rng(21)
    for m, n in ((4, 1), (6, 3), (16, 4), (9, 4)):
        a = rng.standard_normal((m, n))
        cols = [[mpmath.mpf(float(a[i, j])) for i in range(m)] for j in range(n)]
        qs, r_ref = [], [[mpmath.mpf(0)] * n for _ in range(n)]
        for j in range(n):
            v = list(cols[j])
            for k in range(j):
                rkj = mpmath.fsum(qs[k][i] * cols[j][i] for i in range(m))
                r_ref[k][j] = rkj
                v = [v[i] - rkj * qs[k][i] for i in range(m)]
            nv = mpmath.sqrt(mpmath.fsum(x * x for x in v))
            r_ref[j][j] = nv
            qs.append([x / nv for x in v])
        q, r = oracle.cqr2(a)
        rr = np.array([[float(x) for x in row] for row in r_ref])
        qq = np.array([[float(qs[j][i]) for j in range(n)] for i in range(m)])
        assert np.max(np.abs(r - rr)) <= 1e-13 * np.abs(rr).max()
        assert np.max(np.abs(q - qq)) <= 1e-13


def test_cqr2_second_pass_breakdown_offset():
    # An exactly rank-deficient A breaks down in pass 1 with the column index.
    a = gdv_matrix(40, 6, 10.0, 3)
    a[:, 4] = 0.0
    with pytest.raises(oracle.NotSPD) as e:
        oracle.cqr2(a)
    assert e.value.j == 5


def test_mixed_oracle_orthogonality_and_error_level():
    # Mixed form against the FP64 oracle and the orthogonality invariant.
    a = gdv_matrix(4096, 64, 1e3, 1)
    q, r = oracle.cqr2_mixed(a)
    q64, r64 = oracle.cqr2(a)
    assert oracle.orthogonality(q) <= 1e-12
    assert oracle.residual(a, q, r) <= 1e-5       # ~FP32 unit roundoff level
    assert oracle.rel_fro(r, r64) <= 1e-4
    assert oracle.residual(a, q, r) > 1e-12       # really took FP32 arithmetic


# --- FP32 accumulation of the mixed form's pass-1 product (mm_fp32) -----------

def _mm_fp64_sums(a, b):
    """Planted mistake: FP32 operands, but FP64 products and sums, rounded once."""
    a32 = np.asarray(a, np.float64).astype(np.float32).astype(np.float64)
    b32 = np.asarray(b, np.float64).astype(np.float32).astype(np.float64)
    return (a32 @ b32).astype(np.float32)


def _mm_fp16_sums(a, b):
    """Planted mistake: running sums kept in FP16."""
    a32 = np.asarray(a, np.float64).astype(np.float32)
    b32 = np.asarray(b, np.float64).astype(np.float32)
    acc = np.zeros((a32.shape[0], b32.shape[1]), np.float16)
    for k in range(a32.shape[1]):
        acc = (acc.astype(np.float32) + np.outer(a32[:, k], b32[k, :])).astype(np.float16)
    return acc.astype(np.float32)


def _mm_dropped_term(a, b):
    """Planted mistake: the last k term is dropped."""
    a32 = np.asarray(a, np.float64).astype(np.float32)
    b32 = np.asarray(b, np.float64).astype(np.float32)
    return a32[:, :-1] @ b32[:-1, :]


def _order_free_pin(mm) -> bool:
    a, u, rows, signs = fp32_cases.order_free_case()
    q = np.asarray(mm(a, u))
    return bool(np.all(q[rows, fp32_cases.DESIGNED_COL] == signs))


def _accumulation_pins(mm, a, u) -> bool:
    ratio, frac = fp32_cases.fp32_sum_stats(mm(a, u), a, u)
    return ratio <= 1.0 and frac >= 0.2


def _random_product_case(seed=5, m=2000, n=128):
    a = gdv_matrix(m, n, 1e6, seed)
    _, y = oracle.cholinv(oracle.syrk(a))
    return a, y.T.copy()


def test_designed_fp32_sum_is_order_free_and_not_correctly_rounded():
    # brute force over every order and pairing of the three FP32 terms
    for sign in (1.0, -1.0):
        assert fp32_cases.all_fp32_orders_of_designed_sum(sign) == {sign}
        assert fp32_cases.exact_fp32_rounding_of_designed_sum(sign) == sign * (1.0 + 2.0 ** -23)


def test_mm_fp32_designed_case_exact():
    a, u, rows, signs = fp32_cases.order_free_case()
    q = oracle.mm_fp32(a, u)
    assert q.dtype == np.float32
    assert np.all(q[rows, fp32_cases.DESIGNED_COL] == signs)
    # every other entry of these rows is one exact product
    others = [c for c in range(a.shape[1]) if c != fp32_cases.DESIGNED_COL]
    assert np.array_equal(q[np.ix_(rows, others)], a[np.ix_(rows, others)].astype(np.float32))


def test_mm_fp32_single_products_are_correctly_rounded():
    # one nonzero per column of U: each entry is one product, rounded once
    rng = np.random.default_rng(3)
    a = rng.standard_normal((300, 20))
    d = 2.0 ** rng.integers(-3, 4, 20)
    q = oracle.mm_fp32(a, np.diag(d))
    assert np.array_equal(q, (a.astype(np.float32).astype(np.float64) * d).astype(np.float32))


def test_mm_fp32_error_bound_and_fp32_rounding():
    a, u = _random_product_case()
    ratio, frac = fp32_cases.fp32_sum_stats(oracle.mm_fp32(a, u), a, u)
    assert ratio <= 1.0            # within the FP32 summation error bound
    assert frac >= 0.2             # and rounded like FP32 running sums (measured ~0.9)


def test_cqr2_mixed_q1_takes_fp32_sums():
    a = gdv_matrix(3000, 96, 1e5, 8)
    _, _, it = oracle.cqr2_mixed(a, return_intermediates=True)
    assert it["Q1"].dtype == np.float64
    assert np.array_equal(it["Q1"], it["Q1"].astype(np.float32).astype(np.float64))   # stored FP32 values
    assert _accumulation_pins(lambda x, y: it["Q1"], a, it["R1inv"])


@pytest.mark.parametrize("mutant", [_mm_fp64_sums, _mm_fp16_sums, _mm_dropped_term])
def test_pins_catch_planted_fp32_accumulation_mistakes(mutant, monkeypatch):
    assert _order_free_pin(oracle.mm_fp32)
    a, u = _random_product_case()
    assert _accumulation_pins(oracle.mm_fp32, a, u)
    caught = not _order_free_pin(mutant) or not _accumulation_pins(mutant, a, u)
    assert caught
    # planted into the oracle itself, the end-to-end Q1 pin fails too
    monkeypatch.setattr(cqr2_ref, "mm_fp32", mutant)
    a2 = gdv_matrix(3000, 96, 1e5, 8)
    _, _, it = cqr2_ref.cqr2_mixed(a2, return_intermediates=True)
    assert not _accumulation_pins(lambda x, y: it["Q1"].astype(np.float32), a2, it["R1inv"])


# ------------------------------------------------------ planted mistakes ---

def _mutant_cholinv(kind):
    def f(a):
        a = np.asarray(a, dtype=np.float64)
        n = a.shape[0]
        if n == 1:
            if not a[0, 0] > 0:
                raise oracle.NotSPD(1)
            l = math.sqrt(a[0, 0])
            return np.array([[l]]), np.array([[1.0 / l]])
        h = n // 2
        l11, y11 = f(a[:h, :h])
        l21 = a[h:, :h] @ (y11 if kind == "transpose" else y11.T)
        schur = a[h:, h:] - (0.0 if kind == "drop_update" else l21 @ l21.T)
        l22, y22 = f(schur)
        y21 = (y22 @ (l21 @ y11)) if kind == "sign" else -(y22 @ (l21 @ y11))
        l = np.zeros((n, n)); y = np.zeros((n, n))
        l[:h, :h], l[h:, :h], l[h:, h:] = l11, l21, l22
        y[:h, :h], y[h:, :h], y[h:, h:] = y11, y21, y22
        return l, y
    return f


@pytest.mark.parametrize("kind", ["transpose", "drop_update", "sign"])
def test_pins_catch_planted_cholinv_mistakes(kind, monkeypatch):
    mut = _mutant_cholinv(kind)
    d = _gold("cholinv_exact_n8.json")
    try:
        l, y = mut(np.array(d["W"]))
        exact_ok = np.array_equal(l, np.array(d["L"])) and np.array_equal(y, np.array(d["Y"]))
    except oracle.NotSPD:
        exact_ok = False
    assert not exact_ok
    monkeypatch.setattr(cqr2_ref, "cholinv", mut)
    a = gdv_matrix(200, 8, 10.0, 4)
    try:
        q, r = cqr2_ref.cqr2(a)
        qh, rh = oracle.householder_qr_posdiag(a)
        good = oracle.rel_fro(r, rh) <= 1e-9 and oracle.orthogonality(q) <= 1e-12
    except oracle.NotSPD:
        good = False
    assert not good


def test_pins_catch_planted_syrk_mistake(monkeypatch):
    a = integer_matrix(30, 5, 8, 1)
    monkeypatch.setattr(cqr2_ref, "syrk", lambda x: np.asarray(x) @ np.asarray(x).T)
    with pytest.raises(Exception):
        q, r = cqr2_ref.cqr2(a)
        assert r.shape == (5, 5)


def test_pins_catch_planted_second_pass_skip(monkeypatch):
    # Dropping pass 2 (plain CholeskyQR) loses orthogonality at cond 1e6.
    a = gdv_matrix(2000, 32, 1e6, 2)
    q1, r1, _ = oracle.cqr(a)
    assert oracle.orthogonality(q1) > 1e-12


# ---- shifted CholeskyQR3 (the unconditionally stable extension the paper cites) ----

@pytest.mark.parametrize("kappa", [1e10, 1e12])
def test_scqr3_householder_accuracy_where_cqr2_breaks_down(kappa):
    """Past cond ~ u^(-1/2) the Gram matrix is numerically singular: CQR2's
    Cholesky fails, the shifted form stays as accurate as Householder QR."""
    a = gdv_matrix(3000, 40, kappa, 301)
    with pytest.raises(oracle.NotSPD):
        oracle.cqr2(a)
    q, r = oracle.scqr3(a)
    assert np.array_equal(r, np.triu(r)) and np.all(np.diag(r) > 0)
    assert oracle.orthogonality(q) <= 1e-13
    assert oracle.residual(a, q, r) <= 1e-14
    rh = oracle.householder_qr_posdiag(a)[1]
    assert oracle.rel_fro(r, rh) <= 1e-12


@pytest.mark.parametrize("m,n,kappa,seed", [(2000, 30, 1e3, 302), (5000, 64, 1e6, 303)])
def test_scqr3_agrees_with_cqr2_in_its_range(m, n, kappa, seed):
    a = gdv_matrix(m, n, kappa, seed)
    q2, r2 = oracle.cqr2(a)
    q3, r3 = oracle.scqr3(a)
    assert oracle.rel_fro(r3, r2) <= 1e-12
    assert np.max(np.abs(q3 - q2)) <= 1e-9


def test_scqr3_orthonormal_columns_closed_form():
    """A with orthonormal columns: W = I, so R1 = sqrt(1 + s) I and the two
    refinement passes undo the scaling: R = I and Q = A up to a few ulps."""
    h = scipy.linalg.hadamard(256)[:, :24] / 16.0
    q, r = oracle.scqr3(h)
    assert np.max(np.abs(r - np.eye(24))) <= 8 * 2.0 ** -52
    assert np.max(np.abs(q - h)) <= 8 * 2.0 ** -52


def test_scqr3_shift_scales_with_the_gram():
    a = gdv_matrix(500, 10, 1e2, 304)
    w = oracle.syrk(a)
    s = oracle.cholesky_shift(w, 500)
    assert s > 0.0
    assert oracle.cholesky_shift(w * 4.0, 500) == 4.0 * s   # exact: trace and s scale by powers of two


def test_scqr3_power_of_two_scaling_is_exact():
    a = gdv_matrix(1000, 20, 1e12, 305)
    q1, r1 = oracle.scqr3(a)
    q2, r2 = oracle.scqr3(a * 2.0 ** 20)
    assert np.array_equal(q1, q2)
    assert np.array_equal(r1 * 2.0 ** 20, r2)


def test_scqr3_range_ends_near_u_sqrt_mn():
    """The shift keeps pass 1 positive definite, but past cond ~ 1/(u sqrt(mn))
    the shifted Q1 is too ill-conditioned for the refinement and pass 2 breaks
    down (Fukaya et al.'s condition); just inside, it succeeds."""
    a = gdv_matrix(8000, 128, 1e14, 413)
    with pytest.raises(oracle.NotSPD) as e:
        oracle.scqr3(a)
    assert 128 < e.value.j <= 256
    q, r = oracle.scqr3(gdv_matrix(8000, 128, 1e12, 413))
    assert oracle.orthogonality(q) <= 1e-13


def test_scqr3_pins_catch_a_missing_shift(monkeypatch):
    monkeypatch.setattr(cqr2_ref, "cholesky_shift", lambda w, m: 0.0)
    a = gdv_matrix(3000, 40, 1e12, 301)
    with pytest.raises(oracle.NotSPD):
        cqr2_ref.scqr3(a)


# ---- least squares on top of the factorization (x = R^-1 Qᵀ b) ----

@pytest.mark.parametrize("m,n,k,kappa,seed", [(500, 7, 1, 1e2, 501), (3000, 40, 3, 1e4, 502), (2000, 64, 2, 1e6, 503)])
def test_lstsq_matches_lapack_and_is_optimal(m, n, k, kappa, seed):
    a = gdv_matrix(m, n, kappa, seed)
    rng = np.random.default_rng(seed)
    b = a @ rng.standard_normal((n, k)) + 1e-3 * rng.standard_normal((m, k))   # inconsistent system
    x, q, r = oracle.lstsq(a, b)
    x_ref = np.linalg.lstsq(a, b, rcond=None)[0]
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) <= 50 * kappa * 2.0 ** -52 * 100
    # optimality: the residual is orthogonal to range(A)
    res = b - a @ x
    assert np.linalg.norm(a.T @ res) <= 1e3 * 2.0 ** -52 * np.linalg.norm(a) * (
        np.linalg.norm(a) * np.linalg.norm(x) + np.linalg.norm(b))


def test_lstsq_exact_consistent_system():
    """b = A x with A of orthogonal, power-of-two-norm columns: every step is
    exact, so x comes back bit for bit."""
    h = scipy.linalg.hadamard(64)[:, :8] * np.array([1.0, 2.0, 4.0, 0.5, 8.0, 1.0, 2.0, 0.25])
    xt = np.arange(1.0, 9.0)[:, None]
    x, q, r = oracle.lstsq(h, h @ xt)
    assert np.array_equal(x, xt)


# ---- partial inverse (InverseDepth): inverted diagonal blocks + block substitution ----

@pytest.mark.parametrize("n", [5, 8, 13, 16, 33])
@pytest.mark.parametrize("depth", [1, 2, 3])
def test_cholinv_partial_exact_examples(n, depth):
    """On the exact examples every FP64 step is exact, so L must equal the
    exact L bit for bit and every inverted diagonal block must equal the same
    block of the exact L^{-1} (a diagonal block of the inverse of a triangular
    matrix is the inverse of its diagonal block); Y is zero elsewhere."""
    d = _gold(f"cholinv_exact_n{n}.json")
    l, y, blocks = oracle.cholinv_partial(np.array(d["W"]), depth)
    assert np.array_equal(l, np.array(d["L"]))
    y_ex = np.array(d["Y"])
    mask = np.zeros((n, n), dtype=bool)
    assert blocks[0][0] == 0 and blocks[-1][1] == n
    assert all(b0[1] == b1[0] for b0, b1 in zip(blocks, blocks[1:]))
    assert len(blocks) == min(2 ** depth, n) or n < 2 ** depth
    for c0, c1 in blocks:
        assert np.array_equal(y[c0:c1, c0:c1], y_ex[c0:c1, c0:c1])
        mask[c0:c1, c0:c1] = True
    assert np.all(y[~mask] == 0.0)


@pytest.mark.parametrize("m,n,k", [(50, 7, 3), (300, 40, 5)])
def test_solve_right_lt_matches_lapack_trsm(m, n, k):
    """X = B L^{-T} by block substitution against LAPACK's triangular solve."""
    rng = np.random.default_rng(11)
    l = np.tril(rng.standard_normal((n, n))) + 4.0 * np.eye(n)
    blocks = [(0, 2), (2, 3), (3, n // 2), (n // 2, n)]
    y = np.zeros((n, n))
    for c0, c1 in blocks:
        y[c0:c1, c0:c1] = scipy.linalg.solve_triangular(l[c0:c1, c0:c1], np.eye(c1 - c0), lower=True)
    b = rng.standard_normal((m, n))
    x = oracle.solve_right_lt(b, l, y, blocks)
    x_ref = scipy.linalg.solve_triangular(l, b.T, lower=True).T
    assert np.linalg.norm(x - x_ref) <= 1e-13 * np.linalg.norm(x_ref)


def test_cqr2_partial_depth0_is_cqr2():
    a = gdv_matrix(500, 21, 1e4, 12)
    q0, r0 = oracle.cqr2(a)
    q, r = oracle.cqr2_partial(a, 0)
    assert np.array_equal(q, q0) and np.array_equal(r, r0)


@pytest.mark.parametrize("m,n,kappa,seed,depth", [
    (2000, 37, 1e6, 3, 1), (2000, 37, 1e6, 3, 3), (5000, 64, 1e4, 13, 2), (700, 100, 1e6, 14, 4)])
def test_cqr2_partial_matches_householder(m, n, kappa, seed, depth):
    a = gdv_matrix(m, n, kappa, seed)
    q, r = oracle.cqr2_partial(a, depth)
    qh, rh = oracle.householder_qr_posdiag(a)
    assert oracle.orthogonality(q) <= 1e-12
    assert oracle.residual(a, q, r) <= 1e-13
    assert oracle.rel_fro(r, rh) <= 1e-9
    assert np.array_equal(r, np.triu(r)) and np.all(np.diag(r) > 0)


def test_cqr2_partial_power_of_two_scaling_is_exact():
    a = gdv_matrix(400, 24, 1e3, 15)
    q, r = oracle.cqr2_partial(a, 2)
    q2, r2 = oracle.cqr2_partial(a * 2.0 ** 10, 2)
    assert np.array_equal(q2, q) and np.array_equal(r2, r * 2.0 ** 10)


def test_cqr2_partial_breakdown_columns():
    a = gdv_matrix(300, 20, 10.0, 16)
    a[:, 13] = 0.0
    with pytest.raises(oracle.NotSPD) as e:
        oracle.cqr2_partial(a, 2)
    assert e.value.j == 14


@pytest.mark.parametrize("kind", ["sign", "no_transpose", "skip_update"])
def test_pins_catch_planted_block_substitution_mistakes(kind, monkeypatch):
    def mut(b, l, y, blocks):
        b = np.asarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        for c0, c1 in blocks:
            if kind == "sign":
                t = b[:, c0:c1] + x[:, :c0] @ l[c0:c1, :c0].T
            elif kind == "no_transpose":
                t = b[:, c0:c1] - x[:, :c0] @ l[:c0, c0:c1]
            else:
                t = b[:, c0:c1]
            x[:, c0:c1] = t @ y[c0:c1, c0:c1].T
        return x
    d = _gold("cholinv_exact_n13.json")
    monkeypatch.setattr(cqr2_ref, "solve_right_lt", mut)
    try:
        l, y, blocks = cqr2_ref.cholinv_partial(np.array(d["W"]), 2)
        exact_ok = np.array_equal(l, np.array(d["L"]))
    except oracle.NotSPD:
        exact_ok = False
    assert not exact_ok
    a = gdv_matrix(300, 16, 1e3, 17)
    try:
        q, r = cqr2_ref.cqr2_partial(a, 2)
        qh, rh = oracle.householder_qr_posdiag(a)
        good = oracle.rel_fro(r, rh) <= 1e-9 and oracle.orthogonality(q) <= 1e-12
    except oracle.NotSPD:
        good = False
    assert not good
