"""Many problems per launch: cqr2_factor_batched and the continuous-batching
server, against the CPU oracle on the same seeded inputs.

Every problem is held to the single-problem gates (FP64, cond <= 1e6):
||QᵀQ - I||_F <= 1e-12, ||A - QR||_F / ||A||_F <= 1e-13, R within 1e-9 of the
oracle (relative, and elementwise against ||R||_F), Q within 1e-9 elementwise.
Results of a problem in a mix equal its results alone, bit for bit.
"""
import numpy as np
import pytest

import oracle
from synth import gdv_matrix
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_ORTH, TOL_RES, TOL_R, TOL_Q = 1e-12, 1e-13, 1e-9, 1e-9

MIX = [  # (m, n, kappa, seed): every n class, ragged m, chunk boundaries, one tiled-path problem
    (5000, 1, 1.0, 101), (3000, 7, 1e2, 102), (4096, 16, 1e3, 103), (10000, 32, 1e4, 104),
    (777, 33, 1e3, 105), (20000, 64, 1e6, 106), (9000, 100, 1e5, 107), (8193, 128, 1e6, 108),
    (4096 * 3 + 17, 96, 1e4, 109), (128, 128, 1e2, 110), (5000, 200, 1e4, 111), (64, 64, 10.0, 112),
    # 128 < n <= 256 (eight-phase step): 2048-row chunks and a ragged tail, m = n, both blocks ragged
    (3000, 256, 1e5, 116), (2048 * 4 + 1, 129, 1e3, 117), (256, 256, 1e2, 118), (2047, 250, 1e6, 119),
    (6000, 300, 1e3, 120),
    # n >= 512: the tiled path with the blocked look-ahead CholInv (helper streams) from a batched call
    (3000, 600, 1e4, 121),
]


def check(a, q, r, kappa):
    q_ref, r_ref = oracle.cqr2(a)
    assert np.array_equal(r, np.triu(r)) and np.all(np.diag(r) > 0)
    assert oracle.orthogonality(q) <= TOL_ORTH
    assert oracle.residual(a, q, r) <= TOL_RES
    assert oracle.rel_fro(r, r_ref) <= TOL_R
    assert np.max(np.abs(r - r_ref)) <= TOL_R * np.linalg.norm(r_ref)
    if kappa <= 1e6:
        assert np.max(np.abs(q - q_ref)) <= TOL_Q


def test_batched_mix_matches_oracle(gpu_lib):
    import torch
    mats = [gdv_matrix(m, n, k, s) for (m, n, k, s) in MIX]
    infos = torch.full((len(mats),), -5, dtype=torch.int32, device="cuda")
    outs = gpu_lib.factor_batched([to_dev(a) for a in mats], infos)
    assert infos.tolist() == [0] * len(mats)
    for a, (m, n, k, s), (qd, rd) in zip(mats, MIX, outs):
        check(a, to_host(qd), to_host(rd), k)


def test_batched_alone_equals_in_mix(gpu_lib):
    mats = [gdv_matrix(m, n, k, s) for (m, n, k, s) in MIX]
    mixed = gpu_lib.factor_batched([to_dev(a) for a in mats])
    for a, (qm, rm) in zip(mats, mixed):
        (qa, ra), = gpu_lib.factor_batched([to_dev(a)])
        assert np.array_equal(to_host(qa), to_host(qm))
        assert np.array_equal(to_host(ra), to_host(rm))


def test_batched_padded_lda_and_breakdown(gpu_lib):
    import torch
    a1 = gdv_matrix(6001, 48, 1e3, 113)
    a2 = gdv_matrix(3000, 20, 10.0, 114)
    a2[:, 4] = 0.0
    a3 = gdv_matrix(2500, 130, 10.0, 115)
    a3[:, 129] = 0.0              # breakdown in the second diagonal block of the wide CholInv
    a4 = gdv_matrix(3000, 256, 10.0, 116)
    a4[:, 40] = 0.0               # ... and in the first
    a5 = gdv_matrix(4100, 200, 1e4, 117)
    infos = torch.full((5,), -5, dtype=torch.int32, device="cuda")
    outs = gpu_lib.factor_batched([to_dev(a1, ld=6001 + 15), to_dev(a2), to_dev(a3), to_dev(a4),
                                   to_dev(a5, ld=4100 + 9)], infos)
    assert infos.tolist() == [0, 5, 130, 41, 0]
    check(a1, to_host(outs[0][0]), to_host(outs[0][1]), 1e3)
    for k in (1, 2, 3):
        assert np.all(np.isnan(to_host(outs[k][1])))
    check(a5, to_host(outs[4][0]), to_host(outs[4][1]), 1e4)


def _serve(lib, mats, arena, budget=0, max_active=64, arrivals_per_step=3):
    """Submit `mats` a few per step (requests arriving while others run) and
    step until every request is done; returns {tag: (Q, R)} and done order."""
    import torch
    outs = {}
    order = []
    with lib.Server(arena, budget, max_active) as sv:
        sv.clock()
        nxt = 0
        steps = 0
        while len(order) < len(mats):
            for _ in range(arrivals_per_step):
                if nxt < len(mats):
                    A = to_dev(mats[nxt])
                    m, n = mats[nxt].shape
                    Q = lib.empty_colmajor(m, n, device="cuda")
                    R = lib.empty_colmajor(n, n, device="cuda")
                    sv.submit(nxt, A, Q, R)
                    outs[nxt] = (Q, R)
                    nxt += 1
            sv.step()
            for tag, ms in sv.poll():
                assert ms >= 0.0
                order.append(tag)
            steps += 1
            assert steps < 10000
            if nxt == len(mats) and len(order) < len(mats):
                torch.cuda.synchronize()
    assert sorted(order) == list(range(len(mats)))
    return outs, order


def test_server_results_equal_alone(gpu_lib):
    mats = [gdv_matrix(m, n, k, s) for (m, n, k, s) in MIX]
    outs, order = _serve(gpu_lib, mats, arena=256 << 20)
    for i, a in enumerate(mats):
        (qa, ra), = gpu_lib.factor_batched([to_dev(a)])
        q, r = to_host(outs[i][0]), to_host(outs[i][1])
        assert np.array_equal(q, to_host(qa)), i
        assert np.array_equal(r, to_host(ra)), i
        check(a, q, r, MIX[i][2])


def test_server_large_request_reads_after_callers_stream(gpu_lib):
    """A request with n > 256 runs on one of the server's own streams; it must
    still read A only after the caller's earlier work on the server's stream
    (here a spin kernel and then the copy that fills A)."""
    import torch
    m, n = 20000, 300
    a = gdv_matrix(m, n, 1e4, 140)
    src = to_dev(a)
    A = gpu_lib.empty_colmajor(m, n, device="cuda")
    A.zero_()
    Q = gpu_lib.empty_colmajor(m, n, device="cuda")
    R = gpu_lib.empty_colmajor(n, n, device="cuda")
    torch.cuda.synchronize()
    with gpu_lib.Server(256 << 20, 0, 8) as sv:
        sv.clock()
        torch.cuda._sleep(20_000_000)     # keeps the stream busy before A is written
        A.copy_(src)
        sv.submit(0, A, Q, R)
        done = []
        for _ in range(1000):
            sv.step()
            done += sv.poll()
            if done:
                break
            torch.cuda.synchronize()
        assert [t for t, _ in done] == [0]
    check(a, to_host(Q), to_host(R), 1e4)


def test_server_admission_by_footprint(gpu_lib):
    # budget fits about two of these requests: the rest wait in the queue
    mats = [gdv_matrix(20000, 64, 1e3, 120 + i) for i in range(8)]
    foot = 3 * 20000 * 64 * 8 + 64 * 64 * 8
    outs, order = _serve(gpu_lib, mats, arena=64 << 20, budget=int(2.6 * foot), arrivals_per_step=8)
    for i, a in enumerate(mats):
        check(a, to_host(outs[i][0]), to_host(outs[i][1]), 1e3)
    A = to_dev(mats[0])
    Q = gpu_lib.empty_colmajor(20000, 64, device="cuda")
    R = gpu_lib.empty_colmajor(64, 64, device="cuda")
    for arena, budget in ((64 << 10, 0), (64 << 20, 1 << 20)):
        with gpu_lib.Server(arena, budget, 4) as sv:
            with pytest.raises(gpu_lib.CQR2Error) as e:
                sv.submit(0, A, Q, R)      # workspace above the arena / footprint above the budget
            assert e.value.code == gpu_lib.CQR2_ERR_TOO_LARGE


def test_server_slot_limit_one(gpu_lib):
    mats = [gdv_matrix(3000 + 100 * i, 8 * (i + 1), 1e2, 130 + i) for i in range(5)]
    outs, order = _serve(gpu_lib, mats, arena=64 << 20, max_active=1, arrivals_per_step=5)
    assert order == list(range(5))       # one slot: first come, first served
    for i, a in enumerate(mats):
        check(a, to_host(outs[i][0]), to_host(outs[i][1]), 1e2)
