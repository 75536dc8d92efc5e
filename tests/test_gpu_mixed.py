"""CholeskyQR2 with CQR2_MIXED_P1_FP32: pass 1's Q1 = A R1^-1 in FP32
arithmetic (FP32 products and sums, FP32 Q1), Gram, CholInv and pass 2 in FP64.

The paper fixes no precision, so this form has no printed result to match.
It is held to: the orthogonality gate ||QᵀQ - I||_F <= 1e-12 (pass 2 restores
it); the residual and R at the FP32 rounding level against the FP64 oracle,
bounded per condition number; the oracle's own mixed form at the same level
(FP32 sums in a different order); and bitwise equality with the FP64 result
on inputs for which every FP32 operation of pass 1 is exact.
"""
import numpy as np
import pytest

import oracle
from synth import gdv_matrix
from tests import fp32_cases
from synth.matrices import MIXED_KAPPAS
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

MIXED = 1              # CQR2_MIXED_P1_FP32
TOL_ORTH = 1e-12
U32 = 2.0 ** -24
TOL_RES = 200 * U32     # ||A - QR|| / ||A||: fl32(A) alone is a u32-level backward error
TOL_R = 200 * U32       # ||R - R_fp64|| / ||R_fp64||


def mixed_factor(lib, a):
    import torch
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    q, r = lib.factor_ex(to_dev(a), info=info, flags=MIXED)
    return to_host(q), to_host(r), int(info.item())


@pytest.mark.parametrize("m,n,kappa,seed", [
    (4096, 64, 1e3, 51), (20000, 33, 1e6, 52), (262144 // 8, 256, 1e2, 53), (262144 // 8, 256, 1e4, 54),
    (262144 // 8, 256, 1e6, 55), (262144 // 8, 256, 1e7, 56), (3001, 300, 1e5, 57), (1000, 17, 1e3, 58),
    (8192, 520, 1e4, 59),  # n > 256 with m % 4 == 0: the FP32 Q1's Gram takes the direct-copy path
    (10000, 128, 1e4, 60), (7777, 100, 1e6, 61),  # 64 < n <= 128: the 128-column kernels, a ragged tail
])
def test_mixed_gates_against_fp64_oracle(gpu_lib, m, n, kappa, seed):
    a = gdv_matrix(m, n, kappa, seed)
    q, r, info = mixed_factor(gpu_lib, a)
    assert info == 0
    assert np.array_equal(r, np.triu(r)) and np.all(np.diag(r) > 0)
    assert oracle.orthogonality(q) <= TOL_ORTH
    assert oracle.residual(a, q, r) <= TOL_RES
    q_ref, r_ref = oracle.cqr2(a)
    assert oracle.rel_fro(r, r_ref) <= TOL_R
    # against the oracle's mixed form: same precision, other FP32 summation order.
    # Q is conditioned like A (an FP32-level change of R moves Q by ~kappa u32),
    # so Q is compared only where that is small.
    qm, rm = oracle.cqr2_mixed(a)
    assert oracle.rel_fro(r, rm) <= TOL_R
    if kappa <= 1e4:
        assert oracle.rel_fro(q, qm) <= max(TOL_R, 50 * U32 * kappa)


def hadamard_times_bidiagonal(m, n, seed):
    """A = H R with H orthogonal ±1 columns (norm sqrt(m), m a power of 4) and R
    bidiagonal with power-of-two diagonal and ±1 superdiagonal: R^-1 has dyadic
    entries, every FP32 product and partial sum of Q1 = A R1^-1 is exact, and the
    factors are exactly Q = H / sqrt(m), R = sqrt(m) R."""
    rng = np.random.default_rng(seed)
    k = 1
    while k < max(n + 1, 2):
        k *= 2
    h = np.array([[1.0]])
    while h.shape[0] < k:
        h = np.block([[h, h], [h, -h]])
    hcols = np.vstack([h] * (m // k))[:, 1:n + 1]
    d = 2.0 ** rng.integers(-1, 2, n)
    r = np.diag(d) @ (np.eye(n) + np.diag(rng.choice([-1.0, 1.0], n - 1), 1))
    return hcols, r, hcols @ r


@pytest.mark.parametrize("m,n", [(4096, 48), (4096, 200), (16384, 130), (4096, 300)])
def test_mixed_exact_case_bitwise(gpu_lib, m, n):
    hcols, rr, a = hadamard_times_bidiagonal(m, n, 60 + n)
    q, r, info = mixed_factor(gpu_lib, a)
    assert info == 0
    s = np.sqrt(m)
    assert np.array_equal(r, s * rr)
    assert np.array_equal(q, hcols / s)
    qf, rf = gpu_lib.factor(to_dev(a))
    assert np.array_equal(to_host(qf), q) and np.array_equal(to_host(rf), r)


def test_apply_rinv_f32_designed_case_bitwise(gpu_lib):
    """Pass 1's FP32 product alone, on the designed input whose FP32 sums are
    the same in every order and differ from the correctly rounded ones:
    bitwise equal to the oracle's mm_fp32 wherever the result is order-free."""
    col = fp32_cases.DESIGNED_COL
    a, u, rows, signs = fp32_cases.order_free_case()
    q = to_host(gpu_lib.apply_rinv_f32(to_dev(a), to_dev(u)))
    ref = oracle.mm_fp32(a, u)
    assert q.dtype == np.float32
    assert np.all(q[rows, col] == signs)           # FP32 running sums, not 1 + 2^-23
    free = np.ones(q.shape, bool)
    free[:, col] = False
    free[rows, col] = True
    assert np.array_equal(q[free], ref[free])
    # the rest of that column: 4 random terms, order-dependent in FP32
    ratio, _ = fp32_cases.fp32_sum_stats(q, a, u)
    assert ratio <= 1.0


@pytest.mark.parametrize("m,n,seed", [(2000, 128, 71), (4096, 64, 72), (3001, 256, 73), (1000, 300, 74)])
def test_apply_rinv_f32_accumulates_in_fp32(gpu_lib, m, n, seed):
    """On random inputs: within the FP32 summation bound of the exact product,
    rounded like FP32 running sums (most entries differ from the correctly
    rounded product), and within twice that bound of the oracle's mm_fp32."""
    a = gdv_matrix(m, n, 1e6, seed)
    _, y = oracle.cholinv(oracle.syrk(a))
    u = y.T.copy()
    q = to_host(gpu_lib.apply_rinv_f32(to_dev(a), to_dev(u)))
    ratio, frac = fp32_cases.fp32_sum_stats(q, a, u)
    assert ratio <= 1.0
    assert frac >= 0.2
    ref = oracle.mm_fp32(a, u).astype(np.float64)
    a32 = a.astype(np.float32).astype(np.float64)
    u32 = u.astype(np.float32).astype(np.float64)
    bound = n * U32 * (np.abs(a32) @ np.abs(u32)) + 2.0 ** -149
    assert np.all(np.abs(q.astype(np.float64) - ref) <= 2 * bound)


def test_mixed_breakdown_and_determinism(gpu_lib):
    a = gdv_matrix(6000, 40, 10.0, 61)
    q1, r1, i1 = mixed_factor(gpu_lib, a)
    q2, r2, i2 = mixed_factor(gpu_lib, a)
    assert i1 == i2 == 0
    assert np.array_equal(q1, q2) and np.array_equal(r1, r2)
    a[:, 7] = 0.0
    q, r, info = mixed_factor(gpu_lib, a)
    assert info == 8
    assert np.all(np.isnan(r))


def test_mixed_workspace_holds_fp32_q1(gpu_lib):
    m, n = 262144, 256
    w64 = gpu_lib.workspace_size(m, n, 0)
    w32 = gpu_lib.workspace_size(m, n, MIXED)
    assert w32 > 0 and w64 - w32 >= m * n * 4 - 4096


@pytest.mark.slow
@pytest.mark.parametrize("kappa", sorted(MIXED_KAPPAS))
def test_mixed_full_size_kappa_sweep(gpu_lib, kappa):
    """The 262144 x 256 comparison problem at each condition number of the
    sweep, both forms against the FP64 oracle (run with -s to print the row
    of the per-kappa error table)."""
    from synth import workload_matrix
    a = workload_matrix("mixed_262144x256", kappa)
    q, r, info = mixed_factor(gpu_lib, a)
    assert info == 0
    qf, rf = gpu_lib.factor(to_dev(a))
    qf, rf = to_host(qf), to_host(rf)
    q_ref, r_ref = oracle.cqr2(a)
    row = {
        "kappa": kappa,
        "fp64": (oracle.orthogonality(qf), oracle.residual(a, qf, rf), oracle.rel_fro(rf, r_ref),
                 oracle.rel_fro(qf, q_ref)),
        "mixed": (oracle.orthogonality(q), oracle.residual(a, q, r), oracle.rel_fro(r, r_ref),
                  oracle.rel_fro(q, q_ref)),
    }
    print(f"\nkappa {kappa:.0e}  (orth, resid, R rel, Q rel) vs the FP64 oracle: "
          f"FP64 {' '.join(f'{x:.2e}' for x in row['fp64'])} | mixed {' '.join(f'{x:.2e}' for x in row['mixed'])}")
    assert oracle.orthogonality(q) <= TOL_ORTH and oracle.orthogonality(qf) <= TOL_ORTH
    assert oracle.residual(a, q, r) <= TOL_RES
    assert oracle.residual(a, qf, rf) <= 1e-13
    assert oracle.rel_fro(r, r_ref) <= TOL_R
    assert oracle.rel_fro(rf, r_ref) <= 1e-9
