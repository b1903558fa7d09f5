"""The exact constrained minimiser in the normal-equations metric --
TEST INFRASTRUCTURE ONLY.

Section 3.1.1 states the constrained problem as: minimise the norm of
a_fc + A_ff w subject to Q w = B|_F, and its direct solution by the KKT
system whose (1,1) block is A_ff^T A_ff.  Algorithm 1 instead projects in the
Euclidean norm; this module computes the KKT solution for comparison.

Applied to A^T for restriction (as everywhere here), row i of R (C-point i,
F-neighbourhood N) has the block K_i = A[N,N]^T and a_i = A[i,N]^T; the energy
is sum_i |a_i + K_i z_i|^2.  With Abar_i = K_i^T K_i (block diagonal over the
rows), stationarity gives z_i = z_i^0 - Abar_i^{-1} (Q^T lambda)_i, where z^0
is the unconstrained minimiser (the exact local l-AIR solution) and
(Q^T lambda)_i = B_i lambda|_N; the constraints then give the sparse SPD
system  (Q Abar^{-1} Q^T) lambda = Q z^0 - B|_F  over the covered F-points,
whose entry (j, k) is the sum of B_i^2 (Abar_i^{-1})_{jk} over the rows
holding both.  It is assembled row by row and solved directly (SciPy).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import build_R


def kkt_R(n, row_ptr, col_idx, val, cf, B, ell, theta=0.0, strength=None):
    """R (dict as build_R returns) minimising the normal-equations energy
    under R^T B_c = B; also "lam" (n entries, 0 off the covered F-points) and
    "energy" (sum_i |a_i + K_i z_i|^2)."""
    o = build_R(n, row_ptr, col_idx, val, cf, None, ell, theta=theta, strength=strength)
    A = sp.csr_matrix((np.asarray(val, np.float64), np.asarray(col_idx), np.asarray(row_ptr)), shape=(n, n))
    cfa = np.asarray(cf)
    C = np.nonzero(cfa)[0]
    rp, ci = o["row_ptr"], o["col_idx"]
    z0 = np.array(o["val"], np.float64)
    rows = []
    for r, i in enumerate(C):
        e = np.arange(rp[r], rp[r + 1])
        fe = e[ci[e] != i]
        N = ci[fe]
        K = A[N][:, N].toarray().T
        a = A[i, N].toarray().ravel() if len(N) else np.zeros(0)
        rows.append((int(i), fe, N, K, a))
    out = dict(o)
    if B is None:
        out["lam"] = np.zeros(n)
        out["energy"] = sum(float(np.sum((a + K @ z0[fe]) ** 2)) for (_, fe, _, K, a) in rows)
        return out
    Bv = np.asarray(B, np.float64)
    # M = Q Abar^{-1} Q^T and the right-hand side Q z0 - B_F
    Mi, Mj, Mv = [], [], []
    rhs = np.zeros(n)
    covered = np.zeros(n, bool)
    inv = {}
    for (i, fe, N, K, a) in rows:
        if len(N) == 0:
            continue
        Ai = np.linalg.inv(K.T @ K)
        inv[i] = Ai
        jj, kk = np.meshgrid(N, N, indexing="ij")
        Mi.append(jj.ravel())
        Mj.append(kk.ravel())
        Mv.append((Bv[i] ** 2 * Ai).ravel())
        rhs[N] += Bv[i] * z0[fe]
        covered[N] = True
    lam = np.zeros(n)
    idx = np.nonzero(covered & (cfa == 0))[0]
    if len(idx):
        M = sp.coo_matrix((np.concatenate(Mv), (np.concatenate(Mi), np.concatenate(Mj))), shape=(n, n)).tocsr()
        Mc = M[idx][:, idx]
        rhs[idx] -= Bv[idx]
        lam[idx] = spla.spsolve(Mc.tocsc(), rhs[idx])
    z = z0.copy()
    energy = 0.0
    for (i, fe, N, K, a) in rows:
        if len(N) == 0:
            continue
        z[fe] = z0[fe] - Bv[i] * (inv[i] @ lam[N])
        energy += float(np.sum((a + K @ z[fe]) ** 2))
    out["val"] = z
    out["lam"] = lam
    out["energy"] = energy
    return out
