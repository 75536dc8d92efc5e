"""End-to-end CholeskyQR2 on the GPU (cqr2_factor / cqr2_factor_ex) against
the CPU oracle on the same seeded inputs.

Gates (FP64, cond(A) <= 1e6): ||QᵀQ - I||_F <= 1e-12, ||A - QR||_F/||A||_F <= 1e-13,
||R - R_oracle||_F / ||R_oracle||_F <= 1e-9, and element by element
|R - R_oracle| <= 1e-9 ||R_oracle||_F, |Q - Q_oracle| <= 1e-9.
"""
import numpy as np
import pytest

import oracle
from synth import gdv_matrix, integer_matrix, workload_matrix
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_ORTH, TOL_RES, TOL_R, TOL_Q = 1e-12, 1e-13, 1e-9, 1e-9


def check_against_oracle(a, q, r, q_ref, r_ref, kappa=1e6):
    assert np.array_equal(r, np.triu(r))
    assert np.all(np.diag(r) > 0)
    assert oracle.orthogonality(q) <= TOL_ORTH
    assert oracle.residual(a, q, r) <= TOL_RES
    if kappa <= 1e6:
        nr = np.linalg.norm(r_ref)
        assert oracle.rel_fro(r, r_ref) <= TOL_R
        assert np.max(np.abs(r - r_ref)) <= TOL_R * nr
        assert np.max(np.abs(q - q_ref)) <= TOL_Q


@pytest.mark.parametrize("m,n,kappa,seed", [
    (4096, 64, 1e3, 1),        # the 4096 x 64 workload's shape and conditioning
    (4096, 1, 1.0, 2), (4096, 2, 10.0, 3), (1000, 3, 1e2, 4), (777, 7, 1e3, 5),
    (10000, 16, 1e4, 6), (5000, 31, 1e5, 7), (20001, 33, 1e6, 8), (65, 65, 1e2, 9),
    (128, 128, 1e3, 10), (100003, 100, 1e6, 11), (262147, 128, 1e6, 12), (3000, 127, 1e4, 13),
])
def test_factor_matches_oracle(gpu_lib, m, n, kappa, seed):
    a = gdv_matrix(m, n, kappa, seed)
    q_ref, r_ref = oracle.cqr2(a)
    qd, rd = gpu_lib.factor(to_dev(a))
    check_against_oracle(a, to_host(qd), to_host(rd), q_ref, r_ref, kappa)


def test_factor_named_4096x64_workload(gpu_lib):
    a = workload_matrix("tall_4096x64")
    q_ref, r_ref = oracle.cqr2(a)
    qd, rd = gpu_lib.factor(to_dev(a))
    check_against_oracle(a, to_host(qd), to_host(rd), q_ref, r_ref)


@pytest.mark.slow
def test_factor_named_1Mx128_workload_full_size(gpu_lib):
    """The benchmarked 1048576 x 128 (cond 1e6) problem, in the launch
    configuration the benchmark times (cqr2_factor, library workspace)."""
    a = workload_matrix("tall_1Mx128")
    qd, rd = gpu_lib.factor(to_dev(a))
    q, r = to_host(qd), to_host(rd)
    q_ref, r_ref = oracle.cqr2(a)
    check_against_oracle(a, q, r, q_ref, r_ref)


@pytest.mark.slow
def test_factor_named_65536x4096_workload_full_size(gpu_lib):
    """The 65536 x 4096 problem (tiled Gram, recursive CholInv, column-tiled
    Q) in the benchmark's launch configuration, against the oracle on the same
    bytes: R and Q element by element.  Orthogonality and the residual at this
    size are checked on the device with torch's FP64 products (plain library
    GEMMs, not the path under test)."""
    import torch
    a = workload_matrix("rect_65536x4096")
    ad = to_dev(a)
    qd, rd = gpu_lib.factor(ad)
    q, r = to_host(qd), to_host(rd)
    q_ref, r_ref = oracle.cqr2(a)
    assert np.array_equal(r, np.triu(r)) and np.all(np.diag(r) > 0)
    nr = np.linalg.norm(r_ref)
    assert oracle.rel_fro(r, r_ref) <= TOL_R
    assert np.max(np.abs(r - r_ref)) <= TOL_R * nr
    assert np.max(np.abs(q - q_ref)) <= TOL_Q
    qt = qd.contiguous()
    g = qt.t().contiguous() @ qt
    g.diagonal().sub_(1.0)
    assert float(torch.linalg.norm(g)) <= TOL_ORTH
    res = ad.contiguous() - qt @ rd.contiguous()
    assert float(torch.linalg.norm(res) / torch.linalg.norm(ad.contiguous())) <= TOL_RES


@pytest.mark.slow
def test_factor_largest_n(gpu_lib):
    """n = CQR2_MAX_N (16384), nearly square: too large for the oracle, so the
    properties that hold at any size are checked on the device -- upper
    triangular R with a positive diagonal, ||QᵀQ - I||_F and ||A - QR||_F /
    ||A||_F within the first-order bounds (m n + n (n+1)) u and n^2 u of
    CholeskyQR2 -- plus bitwise determinism."""
    import torch
    n = 16384
    m = n + 64
    g = torch.Generator(device="cuda")
    g.manual_seed(901)
    scale = torch.logspace(0, -2, n, dtype=torch.float64, device="cuda")
    ad = (torch.randn((n, m), generator=g, dtype=torch.float64, device="cuda") * scale[:, None]).t()
    q1, r1 = gpu_lib.factor(ad)
    q2, r2 = gpu_lib.factor(ad)
    torch.cuda.synchronize()
    assert torch.equal(q1, q2) and torch.equal(r1, r2)
    u = 2.0 ** -53
    assert bool(torch.all(torch.diagonal(r1) > 0))
    assert bool(torch.all(torch.tril(r1, -1) == 0))
    qt = q1.contiguous()
    gram = qt.t().contiguous() @ qt
    gram.diagonal().sub_(1.0)
    assert float(torch.linalg.norm(gram)) <= (m * n + n * (n + 1)) * u
    res = ad.contiguous() - qt @ r1.contiguous()
    assert float(torch.linalg.norm(res) / torch.linalg.norm(ad.contiguous())) <= n * n * u


def test_factor_lda_padding_and_unaligned(gpu_lib):
    m, n = 9001, 50
    a = gdv_matrix(m, n, 1e4, 21)
    q_ref, r_ref = oracle.cqr2(a)
    for ld, off in ((m + 7, 0), (m + 1, 1), (m, 1)):
        ad = to_dev(a, ld=ld, offset=off)
        qd, rd = gpu_lib.factor(ad)
        check_against_oracle(a, to_host(qd), to_host(rd), q_ref, r_ref)


def test_factor_ex_matches_factor_bitwise(gpu_lib):
    import torch
    a = gdv_matrix(50000, 96, 1e5, 22)
    ad = to_dev(a)
    q1, r1 = gpu_lib.factor(ad)
    info = torch.full((1,), 123, dtype=torch.int32, device="cuda")
    q2, r2 = gpu_lib.factor_ex(ad, info=info)
    assert int(info.item()) == 0
    assert np.array_equal(to_host(q1), to_host(q2))
    assert np.array_equal(to_host(r1), to_host(r2))


def test_factor_deterministic(gpu_lib):
    a = gdv_matrix(300000, 128, 1e6, 23)
    ad = to_dev(a)
    q1, r1 = gpu_lib.factor(ad)
    q1, r1 = to_host(q1), to_host(r1)
    for _ in range(2):
        q2, r2 = gpu_lib.factor(ad)
        assert np.array_equal(q1, to_host(q2))
        assert np.array_equal(r1, to_host(r2))


def test_factor_input_not_modified(gpu_lib):
    a = gdv_matrix(10000, 64, 1e3, 24)
    ad = to_dev(a)
    gpu_lib.factor(ad)
    assert np.array_equal(to_host(ad), a)


def test_factor_power_of_two_scaling_exact(gpu_lib):
    a = gdv_matrix(20000, 40, 1e4, 25)
    q1, r1 = gpu_lib.factor(to_dev(a))
    q2, r2 = gpu_lib.factor(to_dev(a * 2.0 ** -30))
    assert np.array_equal(to_host(q1), to_host(q2))
    assert np.array_equal(to_host(r1) * 2.0 ** -30, to_host(r2))


@pytest.mark.parametrize("j", [0, 9, 63])
def test_factor_breakdown_reports_column(gpu_lib, j):
    import torch
    a = gdv_matrix(5000, 64, 10.0, 26)
    a[:, j] = 0.0
    info = torch.zeros((1,), dtype=torch.int32, device="cuda")
    q, r = gpu_lib.factor_ex(to_dev(a), info=info)
    assert int(info.item()) == j + 1
    assert np.all(np.isnan(to_host(r)))
    with pytest.raises(oracle.NotSPD) as e:
        oracle.cqr2(a)
    assert e.value.j == j + 1


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), float("-inf")])
@pytest.mark.parametrize("n,j", [(64, 17), (128, 100), (200, 150)])
def test_factor_nonfinite_input_reports_column(gpu_lib, bad, n, j):
    """A NaN or infinite entry in column j of A makes row and column j of the
    Gram non-finite; the columns before j factor normally, and pivot j is NaN
    (inf - inf), so pass 1 reports column j + 1 and R is all NaN.  n = 200
    runs the tiled path, where j falls in the second half of the recursion."""
    import torch
    a = gdv_matrix(3000, n, 1e3, 900 + j)
    a[1234, j] = bad
    with np.errstate(invalid="ignore", over="ignore"), pytest.raises(oracle.NotSPD) as e:
        oracle.cqr2(a)
    assert e.value.j == j + 1
    info = torch.zeros((1,), dtype=torch.int32, device="cuda")
    q, r = gpu_lib.factor_ex(to_dev(a), info=info)
    assert int(info.item()) == j + 1
    assert np.all(np.isnan(to_host(r)))


def test_factor_breakdown_without_info_gives_nan_r(gpu_lib):
    a = gdv_matrix(3000, 20, 10.0, 27)
    a[:, 4] = 0.0              # exactly rank deficient: pivot 5 is exactly zero
    q, r = gpu_lib.factor(to_dev(a))
    r = to_host(r)
    with pytest.raises(oracle.NotSPD):
        oracle.cqr2(a)
    assert np.all(np.isnan(r))


def test_factor_n_zero_and_square(gpu_lib):
    import torch
    z = gpu_lib.empty_colmajor(10, 0, device="cuda")
    q, r = gpu_lib.factor(z)
    assert q.shape == (10, 0) and r.shape == (0, 0)
    a = gdv_matrix(96, 96, 1e2, 28)
    q_ref, r_ref = oracle.cqr2(a)
    qd, rd = gpu_lib.factor(to_dev(a))
    check_against_oracle(a, to_host(qd), to_host(rd), q_ref, r_ref)


def test_factor_integer_orthogonal_columns_exact(gpu_lib):
    # Columns orthogonal with power-of-two norms: W is diagonal with exact
    # square roots, so both passes are exact and Q, R are bitwise known.
    h = np.array([[1, 1, 1, 1], [1, -1, 1, -1], [1, 1, -1, -1], [1, -1, -1, 1]], dtype=np.float64)
    a = np.kron(np.ones((256, 1)), h) * np.array([1.0, 2.0, 4.0, 0.5])
    qd, rd = gpu_lib.factor(to_dev(a))
    q, r = to_host(qd), to_host(rd)
    nrm = np.sqrt(1024.0)
    assert np.array_equal(r, np.diag(np.array([1.0, 2.0, 4.0, 0.5]) * nrm))
    assert np.array_equal(q, a / (np.array([1.0, 2.0, 4.0, 0.5]) * nrm))


@pytest.mark.parametrize("m,n,kappa,seed", [
    (2000, 129, 1e3, 31), (10000, 200, 1e5, 32), (30000, 256, 1e6, 33), (1500, 300, 1e4, 34),
    (256, 256, 1e2, 35), (4096, 520, 1e3, 36),
    # n > 1024: R = R2 R1's far-corner tiles take several reduction segments and their sum
    (2500, 1200, 1e3, 37)])
def test_factor_wide_matches_oracle(gpu_lib, m, n, kappa, seed):
    a = gdv_matrix(m, n, kappa, seed)
    q_ref, r_ref = oracle.cqr2(a)
    qd, rd = gpu_lib.factor(to_dev(a))
    check_against_oracle(a, to_host(qd), to_host(rd), q_ref, r_ref, kappa)


def test_factor_wide_breakdown(gpu_lib):
    import torch
    a = gdv_matrix(3000, 256, 10.0, 37)
    a[:, 200] = 0.0
    info = torch.zeros((1,), dtype=torch.int32, device="cuda")
    q, r = gpu_lib.factor_ex(to_dev(a), info=info)
    assert int(info.item()) == 201
    assert np.all(np.isnan(to_host(r)))


@pytest.mark.parametrize("m,n", [(20000, 256), (3000, 1200)])  # 1200: the blocked CholInv on three streams
def test_factor_wide_deterministic(gpu_lib, m, n):
    a = gdv_matrix(m, n, 1e4, 38)
    ad = to_dev(a)
    q1, r1 = gpu_lib.factor(ad)
    q2, r2 = gpu_lib.factor(ad)
    assert np.array_equal(to_host(q1), to_host(q2))
    assert np.array_equal(to_host(r1), to_host(r2))
