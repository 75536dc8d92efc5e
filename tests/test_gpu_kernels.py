"""Parity of each HIP step kernel with the CPU oracle, through the C ABI.

Exactness where the arithmetic allows it (integer-valued data whose sums are
exactly representable: any summation order gives the same bits), otherwise the
standard floating-point error bounds of the operation.
"""
import glob
import json
import math
import os

import numpy as np
import pytest

import oracle
from synth import gdv_matrix, integer_matrix
from tests.gpu_util import U64, gamma, to_dev, to_host

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- Gram ---

@pytest.mark.parametrize("m,n", [(1, 1), (5, 4), (63, 5), (64, 64), (1000, 33), (4113, 128),
                                 (200037, 100), (131072, 128), (77, 3), (300, 17)])
def test_gram_integer_exact(gpu_lib, m, n):
    a = integer_matrix(m, n, 1 << 10, seed=m + n)
    w = to_host(gpu_lib.gram(to_dev(a)))
    assert np.array_equal(w, oracle.syrk(a))


@pytest.mark.parametrize("ld_extra,offset", [(0, 1), (1, 0), (3, 1), (64, 0)])
def test_gram_strided_and_unaligned(gpu_lib, ld_extra, offset):
    m, n = 5000, 45
    a = integer_matrix(m, n, 1 << 9, seed=7)
    w = to_host(gpu_lib.gram(to_dev(a, ld=m + ld_extra, offset=offset)))
    assert np.array_equal(w, oracle.syrk(a))


@pytest.mark.parametrize("m,n,kappa", [(4096, 64, 1e3), (100000, 128, 1e6), (12345, 77, 1e2)])
def test_gram_float_error_bound(gpu_lib, m, n, kappa):
    a = gdv_matrix(m, n, kappa, seed=3)
    w = to_host(gpu_lib.gram(to_dev(a)))
    ref = oracle.syrk(a)
    bound = 2 * gamma(m) * (np.abs(a).T @ np.abs(a))
    assert np.all(np.abs(w - ref) <= bound)
    assert np.array_equal(w, w.T)


@pytest.mark.parametrize("n", [5, 200, 300])
def test_gram_empty_rows(gpu_lib, n):
    a = gpu_lib.empty_colmajor(0, n, device="cuda")
    w = to_host(gpu_lib.gram(a))
    assert np.array_equal(w, np.zeros((n, n)))


# -------------------------------------------------------------- CholInv ---

@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLD, "cholinv_exact_n*.json"))))
def test_cholinv_exact_examples(gpu_lib, path):
    d = json.load(open(path))
    w = np.array(d["W"])
    r, rinv = gpu_lib.cholinv(to_dev(w))
    assert np.array_equal(to_host(r), np.array(d["L"]).T)
    assert np.array_equal(to_host(rinv), np.array(d["Y"]).T)


@pytest.mark.parametrize("n,kappa", [(1, 1.0), (2, 10.0), (7, 1e2), (16, 1e3), (31, 1e3), (64, 1e3),
                                     (100, 1e3), (128, 1e3), (128, 1e1), (33, 1e2)])
def test_cholinv_random_spd(gpu_lib, n, kappa):
    a = gdv_matrix(3 * n + 5, n, kappa, seed=n)
    w = oracle.syrk(a)
    l_ref, y_ref = oracle.cholinv(w)
    r, rinv = gpu_lib.cholinv(to_dev(w))
    r, rinv = to_host(r), to_host(rinv)
    cw = np.linalg.cond(w)
    tol = 20 * n * U64 * cw
    assert oracle.rel_fro(r, l_ref.T) <= tol
    assert oracle.rel_fro(rinv, y_ref.T) <= tol
    assert np.array_equal(r, np.triu(r)) and np.array_equal(rinv, np.triu(rinv))
    assert np.all(np.diag(r) > 0)
    assert np.linalg.norm(r.T @ r - w) <= 10 * n * U64 * np.linalg.norm(w)


def test_cholinv_reads_lower_triangle_only(gpu_lib):
    d = json.load(open(os.path.join(GOLD, "cholinv_exact_n13.json")))
    w = np.array(d["W"])
    polluted = np.tril(w) + np.triu(np.full_like(w, np.nan), 1)
    r, rinv = gpu_lib.cholinv(to_dev(polluted))
    assert np.array_equal(to_host(r), np.array(d["L"]).T)


@pytest.mark.parametrize("j", [0, 5, 12])
def test_cholinv_breakdown_info(gpu_lib, j):
    import torch
    d = json.load(open(os.path.join(GOLD, "cholinv_exact_n13.json")))
    w = np.array(d["W"])
    w[j, :] = 0.0
    w[:, j] = 0.0
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    r, rinv = gpu_lib.cholinv(to_dev(w), info=info)
    assert int(info.item()) == j + 1
    rh = to_host(r)
    assert np.all(np.isnan(rh[np.triu_indices(13)]))
    assert np.all(rh[np.tril_indices(13, -1)] == 0.0)
    with pytest.raises(oracle.NotSPD) as e:
        oracle.cholinv(w)
    assert e.value.j == j + 1


def test_cholinv_nan_pivot(gpu_lib):
    import torch
    w = np.eye(40) * 4.0
    w[17, 17] = np.nan
    info = torch.zeros((1,), dtype=torch.int32, device="cuda")
    gpu_lib.cholinv(to_dev(w), info=info)
    assert int(info.item()) == 18


# ----------------------------------------------------------- apply R^-1 ---

def _int_upper(n, seed, mx=16):
    rng = np.random.default_rng(seed)
    u = np.triu(rng.integers(-mx, mx + 1, size=(n, n)).astype(np.float64))
    return u


@pytest.mark.parametrize("m,n", [(1, 1), (16, 4), (100, 7), (4096, 64), (4099, 128), (70001, 100),
                                 (33, 33), (5000, 32), (129, 65)])
def test_apply_rinv_integer_exact(gpu_lib, m, n):
    a = integer_matrix(m, n, 16, seed=m)
    u = _int_upper(n, seed=n)
    q = to_host(gpu_lib.apply_rinv(to_dev(a), to_dev(u)))
    assert np.array_equal(q, a @ u)


def test_apply_rinv_ignores_lower_triangle_and_in_place(gpu_lib):
    m, n = 3001, 96
    a = integer_matrix(m, n, 16, seed=1)
    u = _int_upper(n, seed=2)
    u_polluted = u + np.tril(np.full((n, n), 1e300), -1)
    ad = to_dev(a, ld=m + 5)
    out = gpu_lib.apply_rinv(ad, to_dev(u_polluted), Q=ad)   # in place
    assert out.data_ptr() == ad.data_ptr()
    assert np.array_equal(to_host(ad), a @ u)


@pytest.mark.parametrize("m,n", [(4096, 64), (50000, 128), (999, 50)])
def test_apply_rinv_float_error_bound(gpu_lib, m, n):
    a = gdv_matrix(m, n, 1e3, seed=5)
    _, _, rinv = oracle.cqr(a)
    q = to_host(gpu_lib.apply_rinv(to_dev(a), to_dev(rinv)))
    ref = a @ rinv
    bound = 2 * gamma(n) * (np.abs(a) @ np.abs(rinv))
    assert np.all(np.abs(q - ref) <= bound)


# -------------------------------------------------------- R = R2 R1 ------

@pytest.mark.parametrize("n", [1, 3, 16, 64, 127, 128])
def test_upper_product_integer_exact(gpu_lib, n):
    r2 = _int_upper(n, seed=10 + n, mx=64)
    r1 = _int_upper(n, seed=20 + n, mx=64)
    r = to_host(gpu_lib.upper_product(to_dev(r2), to_dev(r1)))
    assert np.array_equal(r, oracle.upper_product(r2, r1))


def test_upper_product_float_bound(gpu_lib):
    n = 128
    a = gdv_matrix(1000, n, 1e4, seed=1)
    _, r1, _ = oracle.cqr(a)
    r2 = np.triu(np.eye(n) + 1e-3 * np.random.default_rng(0).standard_normal((n, n)))
    r = to_host(gpu_lib.upper_product(to_dev(r2), to_dev(r1)))
    bound = 2 * gamma(n) * (np.abs(r2) @ np.abs(r1))
    assert np.all(np.abs(r - r2 @ r1) <= bound)
    assert np.array_equal(r, np.triu(r))


# ------------------------------------------------- n > 128 (tiled path) ---

@pytest.mark.parametrize("m,n", [(1000, 129), (5003, 200), (20000, 256), (777, 300),
                                 # n > 256: 128 x 256 tiles, column panels clamped at n, ragged last 16-row chunk
                                 (300, 300), (16, 257), (5, 300), (1000, 700), (4097, 520)])
def test_gram_wide_integer_exact(gpu_lib, m, n):
    a = integer_matrix(m, n, 1 << 8, seed=m + n)
    w = to_host(gpu_lib.gram(to_dev(a)))
    assert np.array_equal(w, oracle.syrk(a))


@pytest.mark.parametrize("m,n", [(300, 129), (1000, 200), (4099, 256), (513, 300)])
def test_apply_rinv_wide_integer_exact(gpu_lib, m, n):
    a = integer_matrix(m, n, 8, seed=m)
    u = _int_upper(n, seed=n, mx=8)
    q = to_host(gpu_lib.apply_rinv(to_dev(a), to_dev(u)))
    assert np.array_equal(q, a @ u)
    ad = to_dev(a)
    gpu_lib.apply_rinv(ad, to_dev(u), Q=ad)      # in place
    assert np.array_equal(to_host(ad), a @ u)


@pytest.mark.parametrize("n", [129, 200, 256])
def test_upper_product_wide_integer_exact(gpu_lib, n):
    r2 = _int_upper(n, seed=1 + n, mx=16)
    r1 = _int_upper(n, seed=2 + n, mx=16)
    r = to_host(gpu_lib.upper_product(to_dev(r2), to_dev(r1)))
    assert np.array_equal(r, oracle.upper_product(r2, r1))


@pytest.mark.parametrize("n,kappa", [(129, 1e2), (200, 1e3), (256, 1e3), (300, 1e2),
                                     # 511: the halving recursion's one-launch products at their largest (n2 = 383)
                                     (511, 1e3),
                                     # n >= 512: the 128-column blocked form on three streams; whole and ragged last blocks
                                     (512, 1e2), (520, 1e2), (640, 1e3), (1000, 1e2), (1153, 1e4)])
def test_cholinv_recursive_random_spd(gpu_lib, n, kappa):
    a = gdv_matrix(2 * n + 7, n, kappa, seed=n)
    w = oracle.syrk(a)
    l_ref, y_ref = oracle.cholinv(w)
    wd = to_dev(w)
    r, rinv = gpu_lib.cholinv(wd)
    r, rinv = to_host(r), to_host(rinv)
    assert np.array_equal(to_host(wd), w)          # input untouched
    cw = np.linalg.cond(w)
    tol = 20 * n * U64 * cw
    assert oracle.rel_fro(r, l_ref.T) <= tol
    assert oracle.rel_fro(rinv, y_ref.T) <= tol
    assert np.array_equal(r, np.triu(r)) and np.array_equal(rinv, np.triu(rinv))
    assert np.all(np.diag(r) > 0)
    assert np.linalg.norm(r.T @ r - w) <= 10 * n * U64 * np.linalg.norm(w)


@pytest.mark.parametrize("n,j", [(256, 3), (256, 150), (256, 255),
                                 # blocked form: first block, a middle block, the ragged last block
                                 (1000, 3), (1000, 500), (1000, 999)])
def test_cholinv_recursive_breakdown(gpu_lib, n, j):
    import torch
    a = gdv_matrix(2 * n + 88, n, 10.0, seed=4)
    w = oracle.syrk(a)
    w[j, :] = 0.0
    w[:, j] = 0.0
    info = torch.zeros((1,), dtype=torch.int32, device="cuda")
    gpu_lib.cholinv(to_dev(w), info=info)
    assert int(info.item()) == j + 1
