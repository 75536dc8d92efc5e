"""Seeded matrix and request generators (host, FP64, column-major).

The paper's experiments use random matrices (Evaluation, Experimental Setup)
whose shapes were only given in figure legends; these generators stand in for
them with controlled condition numbers.  Every matrix is returned as a
Fortran-ordered (column-major) ``numpy.float64`` array with ``lda == m``, so the
bytes handed to the GPU path and to the oracle are identical.

Nothing here performs CholeskyQR arithmetic.  ``numpy.linalg.qr`` (LAPACK
Householder ``geqrf``/``orgqr``) is used only to draw Haar-like orthonormal
factors for ``A = G * D * V``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def _orthonormal(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    """Orthonormal m x n factor of a seeded Gaussian matrix (Householder QR)."""
    g = rng.standard_normal((m, n))
    q, _ = np.linalg.qr(g, mode="reduced")
    return q


def gdv_matrix(m: int, n: int, kappa: float, seed: int) -> np.ndarray:
    """A = G @ diag(logspace(0, -log10(kappa), n)) @ V, column-major FP64.

    G: m x n with orthonormal columns, V: n x n orthogonal, both drawn from
    ``default_rng(seed)`` (G first, then V).  The singular values of A are the
    diagonal of D, so cond_2(A) == kappa up to rounding.
    """
    if m < n or n < 0:
        raise ValueError("need m >= n >= 0")
    rng = np.random.default_rng(seed)
    if n == 0:
        return np.zeros((m, 0), dtype=np.float64, order="F")
    g = _orthonormal(rng, m, n)
    v = _orthonormal(rng, n, n)
    d = np.logspace(0.0, -math.log10(kappa), n) if n > 1 else np.ones(1)
    a = (g * d[None, :]) @ v
    return np.asfortranarray(a)


def scaled_gaussian(m: int, n: int, log10_range: float, seed: int) -> np.ndarray:
    """Entries i.i.d. N(0,1) times column scales logspace(0, -log10_range, n)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, n))
    a *= np.logspace(0.0, -log10_range, n)[None, :]
    return np.asfortranarray(a)


def integer_matrix(m: int, n: int, maxabs: int, seed: int) -> np.ndarray:
    """Integer-valued FP64 matrix with entries in [-maxabs, maxabs].

    With m * maxabs**2 < 2**53 every partial sum of a Gram entry is an exactly
    representable integer, so AᵀA is computed exactly by any summation order.
    """
    rng = np.random.default_rng(seed)
    a = rng.integers(-maxabs, maxabs + 1, size=(m, n)).astype(np.float64)
    return np.asfortranarray(a)


@dataclass(frozen=True)
class Workload:
    name: str
    m: int
    n: int
    kind: str          # "gdv" or "scaled"
    kappa: float
    seed: int
    description: str


# The five workloads the path is measured and tested on.
WORKLOADS = {
    "tall_4096x64": Workload(
        "tall_4096x64", 4096, 64, "gdv", 1e3, 1,
        "A=G*D*V, 4096x64, kappa=1e3"),
    "tall_1Mx128": Workload(
        "tall_1Mx128", 1 << 20, 128, "gdv", 1e6, 2,
        "A=G*D*V, 1048576x128, kappa=1e6"),
    "rect_65536x4096": Workload(
        "rect_65536x4096", 65536, 4096, "scaled", 1e4, 3,
        "N(0,1) times column scales logspace(0,-4,4096), 65536x4096"),
    "mixed_262144x256": Workload(
        "mixed_262144x256", 262144, 256, "gdv", 1e6, 42,
        "A=G*D*V, 262144x256, kappa in {1e2,1e4,1e6,1e7} (seeds 40..43)"),
}

MIXED_KAPPAS = {1e2: 40, 1e4: 41, 1e6: 42, 1e7: 43}


def workload_matrix(name: str, kappa: float | None = None) -> np.ndarray:
    """Matrix of a named workload (optionally another kappa for the mixed sweep)."""
    w = WORKLOADS[name]
    if w.kind == "scaled":
        return scaled_gaussian(w.m, w.n, math.log10(w.kappa), w.seed)
    if kappa is None:
        return gdv_matrix(w.m, w.n, w.kappa, w.seed)
    return gdv_matrix(w.m, w.n, kappa, MIXED_KAPPAS.get(kappa, w.seed))


@dataclass(frozen=True)
class Request:
    idx: int
    m: int
    n: int
    kappa: float
    seed: int
    arrival_s: float


def request_mix(count: int, rate_per_s: float, seed: int,
                m_lo: int = 1024, m_hi: int = 131072,
                ns=(16, 32, 64, 128, 256)) -> list[Request]:
    """Served-stream request list: shapes, conditioning and Poisson arrivals.

    m is log-uniform in [m_lo, m_hi], n uniform over ``ns``, kappa log-uniform
    in [1e1, 1e6]; each request's matrix seed is ``seed * 100003 + i``.
    Inter-arrival gaps are exponential with mean 1/rate (own stream).
    """
    rng = np.random.default_rng(seed)
    arr = np.random.default_rng(seed + 7919)
    t = 0.0
    out = []
    for i in range(count):
        m = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        n = int(ns[rng.integers(0, len(ns))])
        m = max(m, n)
        kappa = 10.0 ** rng.uniform(1.0, 6.0)
        if rate_per_s > 0:
            t += arr.exponential(1.0 / rate_per_s)
        out.append(Request(i, m, n, kappa, seed * 100003 + i, t))
    return out


def gdv_matrix_device(m: int, n: int, kappa: float, seed: int, device="cuda"):
    """A = G diag(logspace(0, -log10 kappa, n)) V generated on a torch device.

    Same construction as ``gdv_matrix`` with torch's seeded generator of that
    device (so the bytes differ from the host version); used where thousands
    of request matrices are needed quickly (the served stream).  G and V are
    the orthonormal factors of seeded Gaussians (torch.linalg.qr).  Returns a
    column-major (strides (1, m)) float64 tensor.
    """
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    g = torch.randn((n, m), generator=gen, device=device, dtype=torch.float64).t()
    g = torch.linalg.qr(g, mode="reduced").Q
    v = torch.randn((n, n), generator=gen, device=device, dtype=torch.float64)
    v = torch.linalg.qr(v, mode="reduced").Q
    d = torch.logspace(0.0, -math.log10(kappa), n, dtype=torch.float64, device=device) if n > 1 else \
        torch.ones(1, dtype=torch.float64, device=device)
    a = (g * d[None, :]) @ v
    out = torch.empty((n, m), dtype=torch.float64, device=device).t()
    out.copy_(a)
    return out
