"""Accuracy measures for QR results (test infrastructure only).

The postconditions of Algorithms 4/5 (A = QR, Q with orthonormal columns, R
upper triangular) turned into numbers, plus a Householder QR whose R is made
positive-diagonal so it can be compared with CholeskyQR2's R (CholeskyQR2 is
as accurate as Householder QR when cond(A) = O(eps^{-1/2}), Introduction).
"""
from __future__ import annotations

import numpy as np


def orthogonality(q: np.ndarray) -> float:
    """||QᵀQ - I||_F."""
    q = np.asarray(q, dtype=np.float64)
    n = q.shape[1]
    return float(np.linalg.norm(q.T @ q - np.eye(n), "fro"))


def residual(a: np.ndarray, q: np.ndarray, r: np.ndarray) -> float:
    """||A - QR||_F / ||A||_F."""
    a = np.asarray(a, dtype=np.float64)
    na = np.linalg.norm(a, "fro")
    if na == 0.0:
        return 0.0
    return float(np.linalg.norm(a - np.asarray(q) @ np.asarray(r), "fro") / na)


def rel_fro(x: np.ndarray, ref: np.ndarray) -> float:
    """||X - Ref||_F / ||Ref||_F."""
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm(np.asarray(x, dtype=np.float64) - ref, "fro")
    nr = np.linalg.norm(ref, "fro")
    return float(d / nr) if nr > 0 else float(d)


def householder_qr_posdiag(a: np.ndarray):
    """LAPACK Householder QR with signs flipped so diag(R) > 0."""
    q, r = np.linalg.qr(np.asarray(a, dtype=np.float64), mode="reduced")
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :], r * s[:, None]
