"""Partial inverse (CQR2_INVERSE_DEPTH) on the GPU against the CPU oracle.

With inverse depth d the top d levels of the CholInv recursion keep only
inverted diagonal blocks and Q is formed by block substitution.  The GPU
recursion splits at multiples of 128 and the oracle at n/2, so the two form
different (equally valid) block sequences: both must meet the FP64 gates and
agree with each other and with the full-inverse factorization, R within 1e-9
and Q within 1e-9 elementwise (cond <= 1e6).
"""
import numpy as np
import pytest

import oracle
from synth import gdv_matrix
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_ORTH, TOL_RES, TOL_R, TOL_Q = 1e-12, 1e-13, 1e-9, 1e-9


def factor(lib, a, depth, ld=None):
    import torch
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    q, r = lib.factor_ex(to_dev(a, ld=ld), info=info, flags=lib.CQR2_INVERSE_DEPTH(depth))
    return to_host(q), to_host(r), int(info.item())


@pytest.mark.parametrize("m,n,kappa,seed,depth", [
    (3000, 200, 1e6, 801, 1),     # n <= 256: blocks 128 + 72 under the tall-skinny kernels
    (20000, 300, 1e6, 802, 1),    # blocks 128 + 172
    (8000, 640, 1e5, 803, 2),     # four blocks
    (5001, 1000, 1e4, 804, 3),    # ragged m, eight blocks (some 128 wide)
    (4000, 520, 1e6, 805, 8),     # depth past the recursion: stops at the 128 base
])
def test_partial_inverse_matches_oracle(gpu_lib, m, n, kappa, seed, depth):
    a = gdv_matrix(m, n, kappa, seed)
    q, r, info = factor(gpu_lib, a, depth)
    assert info == 0
    q_ref, r_ref = oracle.cqr2_partial(a, depth)
    q_full, r_full = oracle.cqr2(a)
    assert np.array_equal(r, np.triu(r)) and np.all(np.diag(r) > 0)
    assert oracle.orthogonality(q) <= TOL_ORTH
    assert oracle.residual(a, q, r) <= TOL_RES
    for rr in (r_ref, r_full):
        assert oracle.rel_fro(r, rr) <= TOL_R
        assert np.max(np.abs(r - rr)) <= TOL_R * np.linalg.norm(rr)
    assert np.max(np.abs(q - q_ref)) <= TOL_Q
    assert np.max(np.abs(q - q_full)) <= TOL_Q


def test_partial_inverse_padded_lda_and_determinism(gpu_lib):
    a = gdv_matrix(6000, 400, 1e5, 810)
    q1, r1, i1 = factor(gpu_lib, a, 2, ld=6000 + 13)
    q2, r2, i2 = factor(gpu_lib, a, 2)
    assert i1 == i2 == 0
    assert np.array_equal(q1, q2) and np.array_equal(r1, r2)
    assert oracle.rel_fro(r1, oracle.cqr2_partial(a, 2)[1]) <= TOL_R


def test_partial_inverse_changes_nothing_at_n_le_128(gpu_lib):
    a = gdv_matrix(9000, 100, 1e5, 811)
    q0, r0, _ = factor(gpu_lib, a, 0)
    q3, r3, _ = factor(gpu_lib, a, 3)
    assert np.array_equal(q0, q3) and np.array_equal(r0, r3)


@pytest.mark.parametrize("n,j,depth", [(300, 250, 1), (640, 130, 2), (640, 5, 2)])
def test_partial_inverse_breakdown_column(gpu_lib, n, j, depth):
    a = gdv_matrix(4000, n, 10.0, 812)
    a[:, j] = 0.0
    q, r, info = factor(gpu_lib, a, depth)
    assert info == j + 1
    assert np.all(np.isnan(r))
