"""Dense brute force on tiny inputs -- TEST INFRASTRUCTURE ONLY.

Everything here is formulated with dense NumPy arrays so that it is an
independent check of the C oracle:

* ``neighbourhoods``: the distance-ell F-neighbourhood of every C-point by
  boolean reachability (no queue, no visited marks), straight from the
  pattern expansion S^{m-1} T of Algorithm 1 applied to M = A^T.  S is the
  classical strength matrix of M: S_xy = 1 for y != x when m_xy != 0 and
  |m_xy| >= theta max_{w != x} |m_xw| (theta = 0: every stored nonzero);
  T = S_fc.  The F-points f with T_fc = 1 form the first hop of column c; each
  further hop adds the F-points x with S_xy = 1 for some y already reached
  (F-point interior vertices).
* ``lair_rows``: per-row local l-AIR solves (Section 2.1, eq. system) with
  ``numpy.linalg.solve``; Remark 1 says the unconstrained algorithm returns
  exactly these rows.
* ``r_ideal``: the ideal restriction [-A_cf A_ff^{-1}, I] (Section 2.1,
  eq. r_ideal) by a dense solve.
* ``product_reference``: a sparse product X Y with its structural pattern
  (every column some product reaches) and a rounding scale per entry, for
  the Galerkin coarse operator R A P (Section 1).
"""
from __future__ import annotations

import numpy as np


def to_dense(n, row_ptr, col_idx, val):
    A = np.zeros((n, n))
    for r in range(n):
        for e in range(row_ptr[r], row_ptr[r + 1]):
            A[r, col_idx[e]] = val[e]
    return A


def strength_transposed(A: np.ndarray, theta: float = 0.0) -> np.ndarray:
    """Classical strength matrix S of M = A^T (boolean, diagonal excluded)."""
    M = A.T
    n = M.shape[0]
    off = ~np.eye(n, dtype=bool)
    mag = np.where(off, np.abs(M), 0.0)
    rowmax = mag.max(axis=1) if n else np.zeros(0)
    return off & (M != 0) & (mag >= theta * rowmax[:, None])


def neighbourhoods(A: np.ndarray, cf: np.ndarray, ell: int, theta: float = 0.0, agg=None):
    """dict C-point -> sorted array of its distance-ell F-neighbourhood.

    agg (optional): the root C-point of every point's aggregate, or -1; then
    T is the aggregation operator (column c = the F-points of c's aggregate)
    instead of S_fc."""
    S = strength_transposed(A, theta).astype(np.int64)
    F = cf == 0
    out = {}
    for c in np.nonzero(cf != 0)[0]:
        if agg is None:
            reach = (S[:, c] > 0) & F  # T = S_fc, column c
        else:
            reach = (np.asarray(agg) == c) & F  # T = aggregation operator, column c
        for _ in range(ell - 1):
            reach = reach | ((S @ reach.astype(np.int64)) > 0) & F
        out[int(c)] = np.nonzero(reach)[0]
    return out


def neighbourhoods_literal(A: np.ndarray, cf: np.ndarray, ell: int, theta: float = 0.0):
    """dict C-point -> sorted F-points of column c of pattern((S^{ell-1} T)|_F)
    taken literally (Algorithm 1's pattern expansion): S the strength matrix
    of A^T with its diagonal, T = [S_fc, I], boolean products.  C-points may
    be interior vertices of a walk here; the searches of this library keep
    F-points only, and the two agree for ell <= 2."""
    n = A.shape[0]
    S = strength_transposed(A, theta) | np.eye(n, dtype=bool)
    F = cf == 0
    C = np.nonzero(cf != 0)[0]
    T = np.zeros((n, n), dtype=bool)
    T[np.ix_(F, C)] = S[np.ix_(F, C)]
    T[C, C] = True
    X = T.astype(np.int64)
    Si = S.astype(np.int64)
    for _ in range(ell - 1):
        X = ((Si @ X) > 0).astype(np.int64)
    return {int(c): np.nonzero((X[:, c] > 0) & F)[0] for c in C}


def lair_rows(A: np.ndarray, cf: np.ndarray, ell: int, theta: float = 0.0, agg=None):
    """Unconstrained rows: dict C-point -> (N, z) with (A[N,N])^T z = -A[i,N]^T."""
    nb = neighbourhoods(A, cf, ell, theta, agg)
    rows = {}
    for i, N in nb.items():
        if len(N) == 0:
            rows[i] = (N, np.zeros(0))
            continue
        M = A[np.ix_(N, N)]
        a = A[i, N]
        rows[i] = (N, np.linalg.solve(M.T, -a))
    return rows


def rows_to_dense_R(rows, cf, n):
    C = np.nonzero(cf != 0)[0]
    R = np.zeros((len(C), n))
    for r, i in enumerate(C):
        N, z = rows[int(i)]
        R[r, N] = z
        R[r, i] = 1.0
    return R


def r_ideal(A: np.ndarray, cf: np.ndarray) -> np.ndarray:
    """R_ideal = [-A_cf A_ff^{-1}, I], returned in the natural (unpermuted) column order."""
    C = np.nonzero(cf != 0)[0]
    F = np.nonzero(cf == 0)[0]
    Acf = A[np.ix_(C, F)]
    Aff = A[np.ix_(F, F)]
    Z = np.linalg.solve(Aff.T, -Acf.T).T
    R = np.zeros((len(C), A.shape[0]))
    R[:, F] = Z
    R[np.arange(len(C)), C] = 1.0
    return R


def csr_to_dense_R(Rrp, Rci, Rva, n):
    m = len(Rrp) - 1
    R = np.zeros((m, n))
    for r in range(m):
        for e in range(Rrp[r], Rrp[r + 1]):
            R[r, Rci[e]] = Rva[e]
    return R


def product_reference(X, Y):
    """Reference for C = X Y (scipy CSR in): (C on the structural pattern, scale).

    The pattern is that of |X| |Y| (no cancellation among non-negative
    products); values are X Y on it (zero where the products cancel); scale
    = (|X| |Y|) entry by entry, the size of the terms of each sum.
    """
    import scipy.sparse as sp

    X = sp.csr_matrix(X)
    Y = sp.csr_matrix(Y)
    S = sp.csr_matrix(abs(X) @ abs(Y))
    S.sort_indices()
    V = sp.csr_matrix(X @ Y)
    vals = np.asarray(V[S.nonzero()]).ravel() if S.nnz else np.zeros(0)
    # S.nonzero() walks rows in order and columns sorted within a row
    C = sp.csr_matrix((vals, S.indices.copy(), S.indptr.copy()), shape=S.shape)
    return C, S
