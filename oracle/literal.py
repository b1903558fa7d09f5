"""Algorithm 1 (C-l-AIR) carried out step by step -- TEST INFRASTRUCTURE ONLY.

Follows Section 3.1.3 in the paper's order, applied to A^T to obtain R
(Section 3.1.3: restriction is Algorithm 1 on the transpose), with every
operator formed explicitly as a dense matrix on tiny problems:

1. tentative operator W^t = -A_fc of A^T, i.e. W^t[f, c] = -a_{c f}, stored
   on the expanded pattern (possibly zero entries);
2. constraint fit: every F-row of W^t is replaced by the minimum-norm
   (pseudo-inverse) solution of  w B_c|_pattern = B_f;
3. block inverses of the local blocks A_ff^{(c)} of A^T: exact, or the
   local diagonal inverse (Section 3.1.2's approximate block inverses; the
   footnote of the comparison with root-node);
4. k iterations of: residual update  w_bar = A_ff^{-1}(-a_fc - A_ff w^t);
   projection  w_bar <- (I - Q^T (Q Q^T)^+ Q) w_bar  with Q assembled entry by
   entry from B_c (Section 3.1, eq. Qdef) and the pseudo-inverse of Q Q^T;
   update  w^t <- w^t + w_bar.

Remark 2 says the result does not change for k > 1 when the inverses are
exact; the tests check that, and that the result equals the closed form the
C oracle evaluates.
"""
from __future__ import annotations

import numpy as np

from . import dense


def _ilu0(K: np.ndarray):
    """Incomplete LU of K without fill: L unit lower, U upper, both on K's
    nonzero pattern; L U agrees with K on that pattern (the defining property,
    Saad, Iterative Methods for Sparse Linear Systems, Section 10.3)."""
    s = K.shape[0]
    P = K != 0
    W = K.astype(np.float64).copy()
    for a in range(1, s):
        for b in range(a):
            if not P[a, b]:
                continue
            W[a, b] /= W[b, b]
            for c in range(b + 1, s):
                if P[a, c]:
                    W[a, c] -= W[a, b] * W[b, c]
    L = np.tril(W, -1) + np.eye(s)
    U = np.triu(W)
    return L, U


def _gmres(K: np.ndarray, r: np.ndarray, m: int) -> np.ndarray:
    """The vector of the Krylov space span{r, K r, ..., K^{m-1} r} that
    minimises ||r - K x|| (what m steps of GMRES from x = 0 return), by an
    orthonormal basis of the space (QR of the Krylov matrix, cut where the
    space stops growing) and a least-squares fit."""
    if not np.any(r):
        return np.zeros_like(r)
    cols = [r / np.linalg.norm(r)]
    for _ in range(m - 1):
        v = K @ cols[-1]
        cols.append(v / np.linalg.norm(v) if np.any(v) else v)
    Q, Rq = np.linalg.qr(np.array(cols).T)
    d = np.abs(np.diag(Rq))
    k = 1
    while k < len(d) and d[k] > 1e-10 * d[0]:
        k += 1
    V = Q[:, :k]
    y = np.linalg.lstsq(K @ V, r, rcond=None)[0]
    return V @ y


def algorithm1_R(A: np.ndarray, cf: np.ndarray, B, ell: int, k: int = 1,
                 fit_constraint: bool = True, theta: float = 0.0, agg=None, inverse: str = "exact",
                 krylov: int = 1):
    """Dense R (n_c x n) from the literal Algorithm 1 on A^T (strength threshold theta).

    inverse: "exact" (the block inverses of step 3), "diag" (the local
    diagonal inverse of each block), "ilu0" (the inverse of each block's
    incomplete LU factors without fill) or "gmres" (`krylov` steps of GMRES
    on each local system from zero).  B = None drops the constraint lines
    (the fit of step 2 and the projection of step 4)."""
    n = A.shape[0]
    At = A.T
    C = [int(i) for i in np.nonzero(cf != 0)[0]]
    nb = dense.neighbourhoods(A, cf, ell, theta, agg)  # pattern of row c of R == column c of W(A^T)
    # stacked unknown vector w*: the nonzeros of W in compressed-column order
    slots = []  # (c, f)
    col_start = {}
    for c in C:
        col_start[c] = len(slots)
        for f in nb[c]:
            slots.append((c, int(f)))
    nw = len(slots)
    constrained = B is not None
    if not constrained:
        B = np.zeros(n)
        fit_constraint = False
    Bm = np.asarray(B, dtype=np.float64).reshape(n, -1)  # k constraint vectors as columns
    kc = Bm.shape[1]
    Bc = {c: Bm[c] for c in C}

    # 1. tentative operator [-A_fc, I] of A^T on the expanded pattern
    wt = np.array([-At[f, c] for (c, f) in slots], dtype=np.float64)

    # Q: k rows per F-point f, entries B_c[t] at the slots (c, f)
    F = [int(f) for f in np.nonzero(cf == 0)[0]]
    frow = {f: r for r, f in enumerate(F)}
    Q = np.zeros((len(F) * kc, nw))
    for s, (c, f) in enumerate(slots):
        Q[frow[f] * kc:(frow[f] + 1) * kc, s] = Bc[c]

    # 2. enforce Q w^t = B|_F row by row: minimum-norm fit of each F-row
    if fit_constraint:
        for f in F:
            idx = [s for s in range(nw) if slots[s][1] == f]
            if not idx:
                continue
            M = np.array([Bc[slots[s][0]] for s in idx]).T  # kc x |idx|
            wt[idx] = np.linalg.pinv(M, rcond=1e-12) @ Bm[f]

    # 3. exact or approximate block inverses of A_ff^{(c)} (of A^T)
    blocks = {}
    inv = {}
    for c in C:
        N = nb[c]
        blocks[c] = At[np.ix_(N, N)]
        if len(N) == 0:
            continue
        if inverse == "exact":
            inv[c] = np.linalg.inv(blocks[c])
        elif inverse == "diag":
            inv[c] = np.diag(1.0 / np.diag(blocks[c]))
        elif inverse == "ilu0":
            L, U = _ilu0(blocks[c])
            inv[c] = np.linalg.inv(U) @ np.linalg.inv(L)
        elif inverse == "gmres":
            inv[c] = None  # applied to each residual below (not a linear map)
        else:
            raise ValueError(inverse)

    if constrained:
        P = np.eye(nw) - Q.T @ np.linalg.pinv(Q @ Q.T, rcond=1e-12) @ Q
    else:
        P = np.eye(nw)
    for _ in range(k):
        wbar = np.zeros(nw)
        for c in C:
            N = nb[c]
            if len(N) == 0:
                continue
            s0 = col_start[c]
            w_c = wt[s0:s0 + len(N)]
            a_fc = At[N, c]
            res = -a_fc - blocks[c] @ w_c
            if inverse == "gmres":
                wbar[s0:s0 + len(N)] = _gmres(blocks[c], res, krylov)
            else:
                wbar[s0:s0 + len(N)] = inv[c] @ res
        wbar = P @ wbar
        wt = wt + wbar

    R = np.zeros((len(C), n))
    for r, c in enumerate(C):
        N = nb[c]
        s0 = col_start[c]
        R[r, N] = wt[s0:s0 + len(N)]
        R[r, c] = 1.0
    return R
