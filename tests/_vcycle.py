"""CPU multigrid harness for the convergence-factor check: test infrastructure.

A hierarchy is built from a restriction builder ``build(A, cf, B, ell) -> R``
(either the oracle or the GPU library):

* R_k = build(A_k, cf_k, B_k, ell);
* P_k = build(A_k^T, cf_k, B_k, ell)^T, i.e. P is formed from A^T the way R is
  formed from A (Section 4.2: for nonsymmetric A, P and R are generated
  separately from A and A^T);
* A_{k+1} = R_k A_k P_k (Galerkin);
* the C-points of every level follow the same geometric rule (every
  ``k``-th node per axis of that level's grid), and B on the coarse level is
  B_c (injection), i.e. ones again;
* direct solve on the coarsest level.

Smoothing (Section 4, basic test framework, and Section 4.2): V(1,1) with
CFF-Jacobi before the coarse correction (one Jacobi sweep on the C-points,
then two on the F-points, weight 1/rho(D^{-1}A), rho estimated by 15 Arnoldi
steps) and FFC-Jacobi without weight after it.

The convergence factor is gamma = (||r_k|| / ||r_0||)^{1/k} (Section 4) for
the stationary V-cycle iteration on A x = 0 from a seeded random start.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def csr_parts(A):
    A = sp.csr_matrix(A)
    A.sum_duplicates()
    A.sort_indices()
    return (A.shape[0], A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64))


def r_from_arrays(n_c, n, rp, ci, va):
    return sp.csr_matrix((va, ci, rp), shape=(n_c, n))


def cf_grid(shape, k):
    grids = np.meshgrid(*[np.arange(s) for s in reversed(shape)], indexing="ij")
    c = np.ones(grids[0].shape, dtype=bool)
    for g in grids:
        c &= (g % k) == 0
    return c.reshape(-1).astype(np.int8)


def arnoldi_rho(M, steps=15, seed=1234):
    """Spectral radius estimate: largest |Ritz value| after `steps` Arnoldi steps."""
    n = M.shape[0]
    m = min(steps, n)
    rng = np.random.default_rng(seed)
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    v = rng.standard_normal(n)
    V[:, 0] = v / np.linalg.norm(v)
    k_used = m
    for j in range(m):
        w = M @ V[:, j]
        for i in range(j + 1):
            H[i, j] = V[:, i] @ w
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] < 1e-14:
            k_used = j + 1
            break
        V[:, j + 1] = w / H[j + 1, j]
    return float(np.max(np.abs(np.linalg.eigvals(H[:k_used, :k_used]))))


class Level:
    def __init__(self, A, cf, shape):
        self.A = sp.csr_matrix(A)
        self.cf = cf.astype(bool)
        self.shape = shape
        self.D = self.A.diagonal()
        self.R = None
        self.P = None
        self.omega = None


def build_hierarchy(A, shape, k, ell, build, min_coarse=64, max_levels=10, build_P=None, galerkin=None):
    """Levels from fine to coarse.  `build(A_csr_parts, cf, B, ell)` returns R as scipy CSR.

    Optional: `build_P(A_csr_parts, cf, B, ell)` returns P directly (else P is
    the transpose of `build` on A^T), and `galerkin(R, A, P)` the coarse
    operator (else R @ A @ P with scipy)."""
    levels = []
    A = sp.csr_matrix(A)
    for _ in range(max_levels):
        cf = cf_grid(shape, k)
        lev = Level(A, cf, shape)
        levels.append(lev)
        if A.shape[0] <= min_coarse or cf.sum() == 0 or cf.sum() == A.shape[0]:
            break
        B = np.ones(A.shape[0])
        lev.R = build(csr_parts(A), cf, B, ell)
        if build_P is None:
            lev.P = sp.csr_matrix(build(csr_parts(A.T), cf, B, ell).T)
        else:
            lev.P = build_P(csr_parts(A), cf, B, ell)
        Dinv = sp.diags(1.0 / lev.D)
        lev.omega = 1.0 / arnoldi_rho(Dinv @ A)
        A = sp.csr_matrix(lev.R @ A @ lev.P) if galerkin is None else galerkin(lev.R, A, lev.P)
        shape = tuple((s + k - 1) // k for s in shape)
    last = levels[-1]
    last.lu = spla.splu(sp.csc_matrix(last.A))
    return levels


def _jacobi(lev, x, b, mask, w):
    r = b - lev.A @ x
    x[mask] += w * r[mask] / lev.D[mask]


def vcycle(levels, x, b, k=0):
    lev = levels[k]
    if k == len(levels) - 1:
        return lev.lu.solve(b)
    C, F = lev.cf, ~lev.cf
    # CFF pre-smoothing, weighted
    _jacobi(lev, x, b, C, lev.omega)
    _jacobi(lev, x, b, F, lev.omega)
    _jacobi(lev, x, b, F, lev.omega)
    r = b - lev.A @ x
    ec = vcycle(levels, np.zeros(lev.R.shape[0]), lev.R @ r, k + 1)
    x = x + lev.P @ ec
    # FFC post-smoothing, no weight
    _jacobi(lev, x, b, F, 1.0)
    _jacobi(lev, x, b, F, 1.0)
    _jacobi(lev, x, b, C, 1.0)
    return x


def convergence_factor(levels, iters=12, seed=7):
    n = levels[0].A.shape[0]
    x = np.random.default_rng(seed).standard_normal(n)
    b = np.zeros(n)
    r0 = np.linalg.norm(levels[0].A @ x)
    for _ in range(iters):
        x = vcycle(levels, x, b)
    rk = np.linalg.norm(levels[0].A @ x)
    return (rk / r0) ** (1.0 / iters)


def oracle_builder():
    import oracle

    def build(parts, cf, B, ell):
        n, rp, ci, va = parts
        o = oracle.build_R(n, rp, ci, va, cf, B, ell)
        return r_from_arrays(o["n_c"], n, o["row_ptr"], o["col_idx"], o["val"])

    return build
