"""Least-squares requests in the continuous-batching server
(cqr2_server_submit_lstsq) mixed with plain QR requests, against the CPU
oracle on the same seeded inputs.

Gates as for cqr2_lstsq: the factorization to the FP64 gates, X within
1e-12 * cond(A) of the oracle's x = R1^-1 R2^-1 Qᵀ b (relative), and the
normal-equations residual at the rounding level.  A request's results in a
mix equal its results served alone, bit for bit.
"""
import numpy as np
import pytest

import oracle
from synth import gdv_matrix
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

# (m, n, nrhs or 0 for a QR request, kappa, seed): every n class, ragged m, one tiled-path problem
MIX = [
    (5000, 1, 1, 1.0, 701), (3000, 7, 0, 1e2, 702), (4096, 16, 3, 1e3, 703), (10000, 32, 0, 1e4, 704),
    (777, 33, 2, 1e3, 705), (20000, 64, 4, 1e6, 706), (9000, 100, 0, 1e5, 707), (8193, 128, 5, 1e6, 708),
    (5000, 200, 2, 1e4, 709), (3000, 300, 0, 1e3, 710), (64, 64, 1, 10.0, 711), (4000, 256, 3, 1e5, 712),
    (3000, 520, 2, 1e3, 713),  # n >= 512: the blocked look-ahead CholInv inside a served solve
]


def _rhs(a, k, seed):
    rng = np.random.default_rng(seed + 5000)
    m, n = a.shape
    return a @ rng.standard_normal((n, k)) + 1e-3 * rng.standard_normal((m, k))


def _serve(lib, reqs, arena=512 << 20, per_step=3):
    """reqs: list of (a, b or None).  Returns {tag: (Q, R, X or None, info)}."""
    import torch
    outs = {}
    done = []
    with lib.Server(arena, 0, 64) as sv:
        sv.clock()
        nxt = 0
        steps = 0
        while len(done) < len(reqs):
            for _ in range(per_step):
                if nxt < len(reqs):
                    a, b = reqs[nxt]
                    m, n = a.shape
                    A = to_dev(a)
                    Q = lib.empty_colmajor(m, n, device="cuda")
                    R = lib.empty_colmajor(n, n, device="cuda")
                    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
                    if b is None:
                        sv.submit(nxt, A, Q, R, info)
                        outs[nxt] = (Q, R, None, info)
                    else:
                        B = to_dev(b)
                        X = lib.empty_colmajor(n, b.shape[1], device="cuda")
                        sv.submit_lstsq(nxt, A, B, X, Q, R, info)
                        outs[nxt] = (Q, R, X, info)
                    nxt += 1
            sv.step()
            done += [t for t, _ in sv.poll()]
            steps += 1
            assert steps < 10000
            if nxt == len(reqs) and len(done) < len(reqs):
                torch.cuda.synchronize()
    assert sorted(done) == list(range(len(reqs)))
    return outs


def _check_lstsq(a, b, q, r, x, kappa):
    x_ref, q_ref, r_ref = oracle.lstsq(a, b)
    assert oracle.orthogonality(q) <= 1e-12
    assert oracle.residual(a, q, r) <= 1e-13
    assert oracle.rel_fro(r, r_ref) <= 1e-9
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) <= 1e-12 * max(kappa, 10.0)
    res = b - a @ x
    assert np.linalg.norm(a.T @ res) <= 1e3 * 2.0 ** -52 * np.linalg.norm(a) * (
        np.linalg.norm(a) * np.linalg.norm(x) + np.linalg.norm(b))


def test_served_lstsq_mix_matches_oracle_and_alone(gpu_lib):
    reqs = []
    for (m, n, k, kappa, seed) in MIX:
        a = gdv_matrix(m, n, kappa, seed)
        reqs.append((a, _rhs(a, k, seed) if k else None))
    outs = _serve(gpu_lib, reqs)
    for i, ((a, b), (m, n, k, kappa, seed)) in enumerate(zip(reqs, MIX)):
        Q, R, X, info = outs[i]
        assert int(info.item()) == 0, i
        q, r = to_host(Q), to_host(R)
        if b is None:
            q_ref, r_ref = oracle.cqr2(a)
            assert oracle.orthogonality(q) <= 1e-12
            assert oracle.rel_fro(r, r_ref) <= 1e-9
            continue
        _check_lstsq(a, b, q, r, to_host(X), kappa)
    # a request served alone gives the same bits as in the mix
    for i in (2, 7, 8):
        alone = _serve(gpu_lib, [reqs[i]])[0]
        for got, ref in zip(alone[:3], outs[i][:3]):
            assert np.array_equal(to_host(got), to_host(ref)), i


def test_served_lstsq_breakdown_gives_nan(gpu_lib):
    a1 = gdv_matrix(3000, 20, 10.0, 720)
    a1[:, 6] = 0.0
    a2 = gdv_matrix(2500, 150, 10.0, 721)
    a2[:, 149] = 0.0
    ok = gdv_matrix(4000, 24, 1e2, 722)
    reqs = [(a1, _rhs(a1, 2, 720)), (ok, _rhs(ok, 3, 722)), (a2, _rhs(a2, 1, 721))]
    outs = _serve(gpu_lib, reqs, per_step=3)
    assert int(outs[0][3].item()) == 7
    assert int(outs[2][3].item()) == 150
    for i in (0, 2):
        assert np.all(np.isnan(to_host(outs[i][2])))
        assert np.all(np.isnan(to_host(outs[i][1])))
    assert int(outs[1][3].item()) == 0
    _check_lstsq(ok, reqs[1][1], to_host(outs[1][0]), to_host(outs[1][1]), to_host(outs[1][2]), 1e2)


def test_served_lstsq_argument_errors(gpu_lib):
    import ctypes
    lib = gpu_lib.load()
    m, n = 1000, 8
    A = to_dev(gdv_matrix(m, n, 10.0, 730))
    B = to_dev(np.ones((m, 2)))
    Q = gpu_lib.empty_colmajor(m, n, device="cuda")
    R = gpu_lib.empty_colmajor(n, n, device="cuda")
    X = gpu_lib.empty_colmajor(n, 2, device="cuda")
    p = gpu_lib.problem(A, Q, R)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    with gpu_lib.Server(16 << 20, 0, 4) as sv:
        h = sv._h
        f = lib.cqr2_server_submit_lstsq
        assert f(None, ctypes.byref(p), ptr(B), m, 2, ptr(X), n, 0) == -1
        assert f(h, None, ptr(B), m, 2, ptr(X), n, 0) == -2
        assert f(h, ctypes.byref(p), None, m, 2, ptr(X), n, 0) == -3
        assert f(h, ctypes.byref(p), ptr(Q), m, 2, ptr(X), n, 0) == -3      # B overlaps Q
        assert f(h, ctypes.byref(p), ptr(B), m - 1, 2, ptr(X), n, 0) == -4
        assert f(h, ctypes.byref(p), ptr(B), m, 0, ptr(X), n, 0) == -5
        assert f(h, ctypes.byref(p), ptr(B), m, 2, None, n, 0) == -6
        assert f(h, ctypes.byref(p), ptr(B), m, 2, ptr(R), n, 0) == -6      # X overlaps R
        assert f(h, ctypes.byref(p), ptr(B), m, 2, ptr(X), n - 1, 0) == -7
        # B may alias A (both only read)
        assert f(h, ctypes.byref(p), ptr(A), m, 2, ptr(X), n, 0) == 0
        sv.step()
        for _ in range(20):
            sv.step()
        import torch
        torch.cuda.synchronize()
        assert [t for t, _ in sv.poll()] == [0]
    x = to_host(X)
    a = to_host(A)
    x_ref, _, _ = oracle.lstsq(a, a[:, :2])
    assert np.allclose(x, x_ref, rtol=0, atol=1e-12)
