"""Least squares on top of the GPU factorization (cqr2_lstsq) against the CPU
oracle's x = R1^-1 R2^-1 Qᵀ b on the same inputs.

X is conditioned like the problem (a change of R at the rounding level moves
X by about cond(A) u relative), so it is held to 1e-12 * cond(A) relative to
the oracle; Q and R to the factorization gates.
"""
import numpy as np
import pytest

import oracle
from synth import gdv_matrix
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,k,kappa,seed", [
    (5000, 1, 1, 1.0, 601), (4096, 16, 3, 1e3, 602), (20000, 64, 1, 1e4, 603), (30011, 128, 5, 1e6, 604),
    (6000, 200, 2, 1e5, 605), (3000, 300, 4, 1e3, 606)])
def test_lstsq_matches_oracle(gpu_lib, m, n, k, kappa, seed):
    a = gdv_matrix(m, n, kappa, seed)
    rng = np.random.default_rng(seed)
    b = a @ rng.standard_normal((n, k)) + 1e-3 * rng.standard_normal((m, k))
    X, Q, R = gpu_lib.lstsq(to_dev(a), to_dev(b))
    x, q, r = to_host(X), to_host(Q), to_host(R)
    x_ref, q_ref, r_ref = oracle.lstsq(a, b)
    assert oracle.orthogonality(q) <= 1e-12
    assert oracle.residual(a, q, r) <= 1e-13
    assert oracle.rel_fro(r, r_ref) <= 1e-9
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) <= 1e-12 * max(kappa, 10.0)
    res = b - a @ x
    assert np.linalg.norm(a.T @ res) <= 1e3 * 2.0 ** -52 * np.linalg.norm(a) * (
        np.linalg.norm(a) * np.linalg.norm(x) + np.linalg.norm(b))


def test_lstsq_exact_consistent_system(gpu_lib):
    import scipy.linalg
    h = scipy.linalg.hadamard(256)[:, :12] * np.array([1.0, 2.0, 4.0, 0.5, 8.0, 1.0, 2.0, 0.25, 1.0, 1.0, 2.0, 4.0])
    xt = np.arange(1.0, 13.0)[:, None] * np.array([[1.0, -2.0]])
    X, _, _ = gpu_lib.lstsq(to_dev(h), to_dev(h @ xt))
    assert np.array_equal(to_host(X), xt)


def test_lstsq_breakdown_gives_nan(gpu_lib):
    import torch
    a = gdv_matrix(3000, 20, 10.0, 610)
    a[:, 3] = 0.0
    info = torch.zeros((1,), dtype=torch.int32, device="cuda")
    X, Q, R = gpu_lib.lstsq(to_dev(a), to_dev(np.ones((3000, 2))), info=info)
    assert int(info.item()) == 4
    assert np.all(np.isnan(to_host(X))) and np.all(np.isnan(to_host(R)))
