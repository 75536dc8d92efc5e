"""cqr2_factor_noalloc: the CholeskyQR2 entry point that allocates nothing
(its workspace is the library's static device array), against cqr2_factor,
the entry point it is a variant of, bit for bit, on two calls in a row (the
second smaller), and against the oracle's gates."""
import numpy as np
import pytest

import oracle
from synth import gdv_matrix
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def test_noalloc_equals_factor_on_consecutive_calls(gpu_lib):
    import torch
    for m, n, kappa, seed in ((300000, 128, 1e6, 201), (5001, 37, 1e3, 202)):
        a = gdv_matrix(m, n, kappa, seed)
        A = to_dev(a)
        Qf, Rf = gpu_lib.factor(A)
        Qn, Rn = gpu_lib.factor_noalloc(A)
        q, r = to_host(Qn), to_host(Rn)
        assert np.array_equal(q, to_host(Qf)), (m, n)
        assert np.array_equal(r, to_host(Rf)), (m, n)
        q_ref, r_ref = oracle.cqr2(a)
        assert oracle.orthogonality(q) <= 1e-12
        assert oracle.residual(a, q, r) <= 1e-13
        assert oracle.rel_fro(r, r_ref) <= 1e-9
        torch.cuda.synchronize()


def test_noalloc_breakdown_and_limit(gpu_lib):
    a = gdv_matrix(4000, 20, 10.0, 203)
    a[:, 6] = 0.0
    _, R = gpu_lib.factor_noalloc(to_dev(a))
    assert np.all(np.isnan(to_host(R)))
    # a problem whose workspace exceeds the static scratch is refused
    big = gpu_lib.empty_colmajor(1 << 20, 200, device="cuda")
    with pytest.raises(gpu_lib.CQR2Error) as e:
        gpu_lib.factor_noalloc(big)
    assert e.value.code == gpu_lib.CQR2_ERR_NOALLOC_LIMIT
