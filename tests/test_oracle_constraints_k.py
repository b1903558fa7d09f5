"""Oracle pins for k > 1 constraint vectors (CPU).

oracle.project_constraints imposes R^T B_c = B for the k columns of B on an
unconstrained R (the Euclidean projection of Algorithm 1 with Q holding k
rows per F-point; Q Q^T block diagonal).  Pinned against:
* k = 1: the closed form of the C oracle's constrained build;
* the literal Algorithm 1 with k constraint vectors (Q assembled entry by
  entry, numpy pseudo-inverse of Q Q^T), including F-columns whose k x k
  Gram matrix is singular (fewer contributing rows than vectors);
* exact constraints on every F-column whose Gram matrix has full rank;
* invariance under an invertible mixing B -> B M of the k vectors (the
  constraint set does not change).
"""
import numpy as np
import pytest

import oracle
from oracle import dense, literal
from paper_2307_00229_amd import problems as P


def _unconstrained(p):
    return oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell)


def _Bk(p, k, seed):
    rng = np.random.default_rng(seed)
    B = rng.uniform(0.5, 1.5, (p.n, k))
    if k > 1:
        B[:, 1] = np.linspace(-1.0, 1.0, p.n) + 0.1 * B[:, 1]  # a second, non-constant mode
    return B


CASES = [
    lambda: P.small_2d(12, stencil=9, eps=0.05, angle=1.0, k=3, ell=2),
    lambda: P.small_2d(14, stencil=5, eps=0.1, angle=0.5, ell=2),
    lambda: P.small_3d(5, eps=0.05, b=(1.0, 0.3, -0.2), ell=2),
    lambda: P.random_sparse(60, 0.06, 5, ell=2, B=None),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_k1_equals_closed_form(case):
    p = CASES[case]()
    B = _Bk(p, 1, case)[:, 0]
    ref = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, B, p.ell)
    got = oracle.project_constraints(_unconstrained(p), p.cf, B)
    assert np.allclose(got["val"], ref["val"], rtol=0, atol=1e-13 * np.abs(ref["val"]).max())
    assert got["n_uncovered"] == ref["n_uncovered"]


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_equals_literal_algorithm1(case, k):
    p = CASES[case]()
    B = _Bk(p, k, 10 + case)
    got = oracle.project_constraints(_unconstrained(p), p.cf, B)
    R = dense.csr_to_dense_R(got["row_ptr"], got["col_idx"], got["val"], p.n)
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    Rl = literal.algorithm1_R(A, p.cf, B, p.ell, k=1)
    assert np.max(np.abs(Rl - R)) <= 1e-11 * np.max(np.abs(R))


@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_constraints_hold_on_full_rank_columns(case, k):
    p = CASES[case]()
    B = _Bk(p, k, 20 + case)
    got = oracle.project_constraints(_unconstrained(p), p.cf, B)
    C = np.nonzero(p.cf)[0]
    rows = np.repeat(np.arange(got["n_c"]), np.diff(got["row_ptr"]))
    fm = got["col_idx"] != C[rows]
    cols = got["col_idx"][fm]
    Bi = B[C[rows[fm]]]
    S = np.zeros((p.n, k))
    G = np.zeros((p.n, k, k))
    np.add.at(S, cols, got["val"][fm][:, None] * Bi)
    np.add.at(G, cols, Bi[:, :, None] * Bi[:, None, :])
    checked = 0
    for j in np.unique(cols):
        w = np.linalg.eigvalsh(G[j])
        if w.min() > 1e-8 * w.max():
            cond = w.max() / w.min()  # the projection's rounding grows with it
            assert np.allclose(S[j], B[j], rtol=0, atol=1e-14 * cond * (1 + np.abs(B[j]).max()))
            checked += 1
    assert checked > 0


@pytest.mark.parametrize("case", range(len(CASES)))
def test_mixing_the_vectors_changes_nothing(case):
    # on every F-column whose Gram matrix has full rank the constraint set is
    # the same for B and B M, and so is the projection (each column is
    # projected on its own); rank-deficient columns are least-squares fits,
    # whose metric M changes
    p = CASES[case]()
    B = _Bk(p, 3, 30 + case)
    M = np.array([[2.0, 0.5, 0.0], [0.0, 1.0, -1.0], [1.0, 0.0, 3.0]])
    a = oracle.project_constraints(_unconstrained(p), p.cf, B)
    b = oracle.project_constraints(_unconstrained(p), p.cf, B @ M)
    C = np.nonzero(p.cf)[0]
    rows = np.repeat(np.arange(a["n_c"]), np.diff(a["row_ptr"]))
    fm = a["col_idx"] != C[rows]
    G = np.zeros((p.n, 3, 3))
    Bi = B[C[rows[fm]]]
    np.add.at(G, a["col_idx"][fm], Bi[:, :, None] * Bi[:, None, :])
    full = np.array([np.linalg.eigvalsh(G[j]).min() > 1e-6 * np.linalg.eigvalsh(G[j]).max() for j in range(p.n)])
    sel = fm & full[a["col_idx"]]
    assert sel.sum() > 0
    assert np.allclose(a["val"][sel], b["val"][sel], rtol=0, atol=1e-10 * np.abs(a["val"]).max())
