"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This package only draws random matrices and request mixes; it contains none of
the factorization's arithmetic.  See ``synth.matrices``.
"""
from .matrices import (  # noqa: F401
    WORKLOADS,
    gdv_matrix,
    gdv_matrix_device,
    integer_matrix,
    request_mix,
    scaled_gaussian,
    workload_matrix,
)
