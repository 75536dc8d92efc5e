"""Shifted CholeskyQR3 on the GPU (CQR2_SHIFTED_CQR3) against the CPU oracle.

Inside CholeskyQR2's range (cond <= 1e6) the FP64 gates hold against the
oracle's shifted form; far past it (cond 1e10 .. 1e14, where CholeskyQR2
breaks down) orthogonality, residual and R against Householder QR still
hold at the FP64 level.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
from synth import gdv_matrix, workload_matrix
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

SHIFTED = 2
TOL_ORTH, TOL_RES, TOL_R, TOL_Q = 1e-12, 1e-13, 1e-9, 1e-9


def shifted_factor(lib, a, ld=None):
    import torch
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    q, r = lib.factor_ex(to_dev(a, ld=ld), info=info, flags=SHIFTED)
    return to_host(q), to_host(r), int(info.item())


@pytest.mark.parametrize("m,n,kappa,seed", [
    (4096, 1, 1.0, 401), (3000, 17, 1e3, 402), (20000, 64, 1e6, 403), (10007, 100, 1e4, 404),
    (50000, 128, 1e6, 405), (5000, 200, 1e5, 406), (30000, 256, 1e6, 407), (2000, 300, 1e3, 408),
])
def test_shifted_matches_oracle(gpu_lib, m, n, kappa, seed):
    a = gdv_matrix(m, n, kappa, seed)
    q, r, info = shifted_factor(gpu_lib, a)
    assert info == 0
    q_ref, r_ref = oracle.scqr3(a)
    assert np.array_equal(r, np.triu(r)) and np.all(np.diag(r) > 0)
    assert oracle.orthogonality(q) <= TOL_ORTH
    assert oracle.residual(a, q, r) <= TOL_RES
    assert oracle.rel_fro(r, r_ref) <= TOL_R
    assert np.max(np.abs(r - r_ref)) <= TOL_R * np.linalg.norm(r_ref)
    assert np.max(np.abs(q - q_ref)) <= TOL_Q


@pytest.mark.slow
def test_shifted_named_1Mx128_workload_full_size(gpu_lib):
    """The 1048576 x 128 (cond 1e6) problem that `bench.py --shifted` times, in
    the same launch configuration (factor_ex with the shifted flag)."""
    a = workload_matrix("tall_1Mx128")
    q, r, info = shifted_factor(gpu_lib, a)
    assert info == 0
    q_ref, r_ref = oracle.scqr3(a)
    assert np.array_equal(r, np.triu(r)) and np.all(np.diag(r) > 0)
    assert oracle.orthogonality(q) <= TOL_ORTH
    assert oracle.residual(a, q, r) <= TOL_RES
    assert oracle.rel_fro(r, r_ref) <= TOL_R
    assert np.max(np.abs(q - q_ref)) <= TOL_Q


@pytest.mark.parametrize("m,n,kappa,seed", [(6000, 40, 1e10, 411), (20000, 96, 1e12, 412),
                                            (8000, 128, 1e12, 413), (12000, 256, 1e12, 414)])
def test_shifted_far_past_cqr2_range(gpu_lib, m, n, kappa, seed):
    import torch
    a = gdv_matrix(m, n, kappa, seed)
    # plain CholeskyQR2 fails here: its Cholesky breaks down, or it loses orthogonality
    info = torch.zeros((1,), dtype=torch.int32, device="cuda")
    q2, _ = gpu_lib.factor_ex(to_dev(a), info=info)
    assert int(info.item()) != 0 or oracle.orthogonality(to_host(q2)) > TOL_ORTH
    q, r, info3 = shifted_factor(gpu_lib, a)
    assert info3 == 0
    assert oracle.orthogonality(q) <= TOL_ORTH
    assert oracle.residual(a, q, r) <= TOL_RES
    rh = oracle.householder_qr_posdiag(a)[1]
    assert oracle.rel_fro(r, rh) <= 1e-10
    _, r_ref = oracle.scqr3(a)
    assert oracle.rel_fro(r, r_ref) <= 1e-10


def test_shifted_breakdown_beyond_its_range(gpu_lib):
    """Past cond ~ 1 / (u sqrt(m n)) the shifted form breaks down too, in its
    second pass, on the GPU as in the oracle (the column may differ: the
    pivot there is zero to working precision)."""
    a = gdv_matrix(8000, 128, 1e14, 413)
    with pytest.raises(oracle.NotSPD) as e:
        oracle.scqr3(a)
    assert 128 < e.value.j <= 256
    q, r, info = shifted_factor(gpu_lib, a)
    assert 128 < info <= 256
    assert np.all(np.isnan(r))


def test_shifted_orthonormal_columns_closed_form(gpu_lib):
    h = scipy.linalg.hadamard(4096)[:, 1:97] / 64.0
    q, r, info = shifted_factor(gpu_lib, h)
    assert info == 0
    assert np.max(np.abs(r - np.eye(96))) <= 16 * 2.0 ** -52
    assert np.max(np.abs(q - h)) <= 16 * 2.0 ** -52


@pytest.mark.parametrize("n", [48, 160])
def test_shifted_power_of_two_scaling_and_determinism(gpu_lib, n):
    a = gdv_matrix(9000, n, 1e12, 420 + n)
    q1, r1, _ = shifted_factor(gpu_lib, a)
    q2, r2, _ = shifted_factor(gpu_lib, a * 2.0 ** -24, ld=9000 + 3)
    q3, r3, _ = shifted_factor(gpu_lib, a)
    assert np.array_equal(q1, q3) and np.array_equal(r1, r3)
    assert np.array_equal(q1, q2)
    assert np.array_equal(r1 * 2.0 ** -24, r2)


@pytest.mark.parametrize("n,j", [(30, 11), (140, 0)])
def test_shifted_zero_column_breaks_down_in_second_pass(gpu_lib, n, j):
    """The shift keeps pass 1 positive definite; the zero column of Q1 then
    stops pass 2 at its column, reported as n + j (oracle and GPU alike)."""
    a = gdv_matrix(4000, n, 10.0, 430 + n)
    a[:, j] = 0.0
    with pytest.raises(oracle.NotSPD) as e:
        oracle.scqr3(a)
    q, r, info = shifted_factor(gpu_lib, a)
    assert info == e.value.j == n + j + 1
    assert np.all(np.isnan(r))


@pytest.mark.parametrize("n", [40, 200])
def test_shifted_ignores_stale_output_contents(gpu_lib, n):
    """R (and the workspace) may hold anything on entry, NaN included: the
    triangular products read only their declared triangles."""
    import torch
    a = gdv_matrix(5000, n, 1e6, 440)
    Q = gpu_lib.empty_colmajor(5000, n, device="cuda")
    R = gpu_lib.empty_colmajor(n, n, device="cuda")
    R.fill_(float("nan"))
    wb = gpu_lib.workspace_size(5000, n, SHIFTED)
    work = torch.full((wb // 8 + 1,), float("nan"), dtype=torch.float64, device="cuda")
    q, r = gpu_lib.factor_ex(to_dev(a), Q=Q, R=R, work=work, flags=SHIFTED)
    q, r = to_host(q), to_host(r)
    q_ref, r_ref = oracle.scqr3(a)
    assert oracle.rel_fro(r, r_ref) <= TOL_R
    assert oracle.residual(a, q, r) <= TOL_RES
