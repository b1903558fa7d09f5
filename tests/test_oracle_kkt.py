"""Oracle pins for the normal-equations (KKT) minimiser (CPU).

oracle.kkt.kkt_R solves Section 3.1.1's constrained problem exactly through
the Schur complement Q Abar^{-1} Q^T.  Pinned against:
* the KKT system of Section 3.1.1 assembled entry by entry (Abar block
  diagonal with K_i^T K_i, Q from B_c) and solved densely on tiny problems;
* the optimality conditions themselves: K_i^T (K_i z_i + a_i) + B_i lambda|_N
  = 0 on every row, and the constraints;
* Algorithm 1's Euclidean projection where the two metrics coincide: when
  every K_i is a multiple of the identity (5-point grid, distance 1, constant
  coefficients) Abar_i is too, and the minimisers agree;
* its own definition: no feasible R has a lower energy, in particular not
  the Euclidean projection.
"""
import numpy as np
import pytest

import oracle
from oracle import dense, kkt
from paper_2307_00229_amd import problems as P

CASES = [
    lambda: P.small_2d(8, stencil=9, eps=0.05, angle=1.0, k=3, ell=2),
    lambda: P.small_2d(10, stencil=5, eps=0.1, angle=0.5, ell=2),
    lambda: P.small_3d(4, eps=0.05, b=(1.0, 0.3, -0.2), ell=2),
    lambda: P.random_sparse(40, 0.08, 5, ell=2),
]


def _blocks(p):
    """(i, N, K, a) per C-point from the dense matrix and the oracle pattern."""
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    nb = dense.neighbourhoods(A, p.cf, p.ell)
    return A, [(int(i), np.asarray(nb[i], int), A[np.ix_(nb[i], nb[i])].T, A[i, nb[i]]) for i in np.nonzero(p.cf)[0]]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_equals_the_assembled_kkt_system(case):
    p = CASES[case]()
    A, blocks = _blocks(p)
    slots = [(i, int(f)) for (i, N, _, _) in blocks for f in N]
    nw = len(slots)
    F = sorted({f for (_, f) in slots})
    G = np.zeros((nw, nw))
    g = np.zeros(nw)
    s0 = 0
    for (i, N, K, a) in blocks:
        s = len(N)
        G[s0:s0 + s, s0:s0 + s] = K.T @ K
        g[s0:s0 + s] = -K.T @ a
        s0 += s
    Q = np.zeros((len(F), nw))
    for t, (i, f) in enumerate(slots):
        Q[F.index(f), t] = p.B[i]
    KKT = np.block([[G, Q.T], [Q, np.zeros((len(F), len(F)))]])
    sol = np.linalg.solve(KKT, np.concatenate([g, p.B[F]]))
    got = kkt.kkt_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)
    R = dense.csr_to_dense_R(got["row_ptr"], got["col_idx"], got["val"], p.n)
    C = list(np.nonzero(p.cf)[0])
    Rk = np.zeros_like(R)
    for t, (i, f) in enumerate(slots):
        Rk[C.index(i), f] = sol[t]
    for r, i in enumerate(C):
        Rk[r, i] = 1.0
    assert np.max(np.abs(Rk - R)) <= 1e-9 * np.abs(R).max()


@pytest.mark.parametrize("case", range(len(CASES)))
def test_optimality_conditions(case):
    p = CASES[case]()
    A, blocks = _blocks(p)
    got = kkt.kkt_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)
    R = dense.csr_to_dense_R(got["row_ptr"], got["col_idx"], got["val"], p.n)
    lam = got["lam"]
    C = list(np.nonzero(p.cf)[0])
    for (i, N, K, a) in blocks:
        if len(N) == 0:
            continue
        z = R[C.index(i), N]
        grad = K.T @ (K @ z + a) + p.B[i] * lam[N]
        assert np.abs(grad).max() <= 1e-8 * max(1.0, np.abs(K.T @ a).max())
    Fc = [f for f in range(p.n) if p.cf[f] == 0 and np.any(R[:, f])]
    colsum = (R[:, Fc] * p.B[C][:, None]).sum(axis=0)
    assert np.allclose(colsum, p.B[Fc], rtol=0, atol=1e-10 * np.abs(p.B).max())


def test_equals_the_euclidean_projection_when_every_block_is_a_multiple_of_I():
    p = P.cfg1()  # 5-point, distance 1, C = (even, even), constant coefficients
    got = kkt.kkt_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)
    ref = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)
    assert np.allclose(got["val"], ref["val"], rtol=0, atol=1e-12 * np.abs(ref["val"]).max())


@pytest.mark.parametrize("case", range(len(CASES)))
def test_no_feasible_r_has_lower_energy(case):
    p = CASES[case]()
    A, blocks = _blocks(p)
    C = list(np.nonzero(p.cf)[0])

    def energy(o):
        R = dense.csr_to_dense_R(o["row_ptr"], o["col_idx"], o["val"], p.n)
        return sum(float(np.sum((a + K @ R[C.index(i), N]) ** 2)) for (i, N, K, a) in blocks)

    got = kkt.kkt_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)
    euc = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)
    assert energy(got) <= energy(euc) * (1 + 1e-12)
    assert abs(energy(got) - got["energy"]) <= 1e-9 * max(1.0, got["energy"])
    # any feasible perturbation (zero column sums of B_i d_ij) raises it
    rng = np.random.default_rng(case)
    base = np.array(got["val"])
    rows = np.repeat(np.arange(got["n_c"]), np.diff(got["row_ptr"]))
    Cn = np.array(C)
    fm = got["col_idx"] != Cn[rows]
    for _ in range(3):
        d = np.zeros_like(base)
        d[fm] = rng.standard_normal(fm.sum())
        Bi = p.B[Cn[rows]]
        s = np.zeros(p.n)
        w = np.zeros(p.n)
        np.add.at(s, got["col_idx"][fm], d[fm] * Bi[fm])
        np.add.at(w, got["col_idx"][fm], Bi[fm] ** 2)
        d[fm] -= Bi[fm] * s[got["col_idx"][fm]] / w[got["col_idx"][fm]]  # project onto Q d = 0
        pert = dict(got)
        pert["val"] = base + 1e-3 * d
        assert energy(pert) >= got["energy"] * (1 - 1e-12)


def test_without_B_is_the_unconstrained_build():
    p = CASES[1]()
    got = kkt.kkt_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell)
    ref = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell)
    assert np.array_equal(got["val"], ref["val"])
