"""CPU FP64 oracle for CholeskyQR2 (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU product path never calls it, and it shares no
code with the HIP kernels or their host runtime.
"""
from .cqr2_ref import (  # noqa: F401
    NotSPD,
    cholinv,
    cholinv_partial,
    cqr,
    cqr_partial,
    cqr2_partial,
    solve_right_lt,
    cqr2,
    cqr2_mixed,
    mm_fp32,
    cholesky_shift,
    scqr3,
    lstsq,
    syrk,
    upper_product,
)
from .checks import (  # noqa: F401
    orthogonality,
    residual,
    rel_fro,
    householder_qr_posdiag,
)
