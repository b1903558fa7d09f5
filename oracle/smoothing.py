"""Smoothing of the constraint vector B -- TEST INFRASTRUCTURE ONLY.

Section 4 (basic test framework and solver parameters) pre-smooths the mode
constraint vector B = 1 on every level with iterations of CFF-weighted
Jacobi: per iteration one weighted Jacobi sweep on the C-points, then two on
the F-points, applied to the homogeneous system M x = 0 (so smooth error is
what remains).  The weight is an input here (the paper takes 1/rho(D^{-1}A)).

For interpolation M = A; the restriction is built from A^T (Section 3.1.3),
whose constraint vector is smoothed with M = A^T.

A sweep on a subset S updates every i in S from the same old x:
    x_i <- x_i - omega * (M x)_i / m_ii,   i in S;   other entries unchanged.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def jacobi_subset(M, x, mask, omega):
    """One weighted Jacobi sweep for M x = 0 on the points where mask is true."""
    M = sp.csr_matrix(M)
    d = M.diagonal()
    r = -(M @ x)
    out = x.copy()
    out[mask] = x[mask] + omega * r[mask] / d[mask]
    return out


def cff_jacobi(A, cf, B, iterations, omega, transpose=False):
    """B after `iterations` CFF-weighted-Jacobi iterations on A (or A^T)."""
    M = sp.csr_matrix(A.T if transpose else A)
    C = np.asarray(cf) != 0
    F = ~C
    x = np.array(B, dtype=np.float64, copy=True)
    for _ in range(iterations):
        x = jacobi_subset(M, x, C, omega)
        x = jacobi_subset(M, x, F, omega)
        x = jacobi_subset(M, x, F, omega)
    return x
