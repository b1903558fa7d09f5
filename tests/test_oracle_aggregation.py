"""Oracle pins for the aggregation-based base pattern (CPU only).

With aggregation-based coarsening, Algorithm 1 (Section 3.1.3 and its
footnote on the aggregation operator) takes T = the aggregation operator:
column c holds the points of c's aggregate, and the pattern is S^{m-1} T.
The C oracle lists each root's F-members and expands them ell-1 times.
Pinned against: the aggregates themselves at ell = 1, a hand example, the
literal dense S^{m-1} T, dense solves of the unconstrained rows and the
literal Algorithm 1 with the constraint.
"""
import numpy as np
import pytest

import oracle
from oracle import dense, literal
from paper_2307_00229_amd import problems as P


def _pats(p, theta=0.0, B=None):
    o = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, B, p.ell, theta=theta, agg=p.agg)
    C = np.nonzero(p.cf)[0]
    return {int(i): [int(c) for c in o["col_idx"][o["row_ptr"][r]:o["row_ptr"][r + 1]] if c != i]
            for r, i in enumerate(C)}, o


CASES = [
    lambda ell: P.greedy_aggregates(P.small_2d(14, stencil=5, eps=0.1, angle=0.5, ell=ell)),
    lambda ell: P.greedy_aggregates(P.small_2d(12, stencil=9, eps=1e-3, angle=2.0, ell=ell)),
    lambda ell: P.greedy_aggregates(P.small_3d(6, eps=0.05, b=(1.0, 0.3, -0.2), ell=ell)),
    lambda ell: P.greedy_aggregates(P.random_sparse(60, 0.06, 13, ell=ell, B=None)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_distance_one_pattern_is_the_aggregate(case):
    p = CASES[case](1)
    pats, _ = _pats(p)
    for c, cols in pats.items():
        members = [j for j in range(p.n) if p.agg[j] == c and p.cf[j] == 0]
        assert cols == members


def test_hand_example():
    # path 0 - 1 - 2 - 3 - 4 (symmetric tridiagonal); aggregates {0: 0, 1},
    # {3: 2, 3, 4}; ell = 2: row 0 = {1} + one step from 1 = {1, 2};
    # row 3 = {2, 4} + one step = {1, 2, 4}
    n = 5
    A = np.diag(np.full(n, 2.0)) + np.diag(np.full(n - 1, -1.0), 1) + np.diag(np.full(n - 1, -1.0), -1)
    rp, ci, va = [0], [], []
    for r in range(n):
        cols = np.nonzero(A[r])[0]
        ci += cols.tolist()
        va += A[r, cols].tolist()
        rp.append(len(ci))
    cf = np.array([1, 0, 0, 1, 0], np.int8)
    agg = np.array([0, 0, 3, 3, 3], np.int32)
    p = P.Problem("path5", n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va), cf, None, 2, agg=agg)
    pats, _ = _pats(p)
    assert pats == {0: [1, 2], 3: [1, 2, 4]}


def test_points_outside_any_aggregate():
    p = CASES[0](1)
    agg = p.agg.copy()
    F = np.nonzero(p.cf == 0)[0]
    agg[F[0]] = -1          # unaggregated
    agg[F[1]] = F[2]        # an F-point is no root
    agg[F[3]] = p.n + 5     # out of range
    q = P.Problem(p.name, p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, 1, agg=agg)
    pats, _ = _pats(q)
    allcols = set(c for cols in pats.values() for c in cols)
    assert F[0] not in allcols and F[1] not in allcols and F[3] not in allcols


@pytest.mark.parametrize("theta", [0.0, 0.25])
@pytest.mark.parametrize("ell", [1, 2, 3])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_pattern_equals_literal_expansion(case, ell, theta):
    p = CASES[case](ell)
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    pats, _ = _pats(p, theta)
    nb = dense.neighbourhoods(A, p.cf, ell, theta, p.agg)
    assert pats == {i: v.tolist() for i, v in nb.items()}


@pytest.mark.parametrize("case", range(len(CASES)))
def test_rows_equal_dense_solves(case):
    p = CASES[case](2)
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    rows = dense.lair_rows(A, p.cf, 2, 0.0, p.agg)
    _, o = _pats(p)
    R = dense.csr_to_dense_R(o["row_ptr"], o["col_idx"], o["val"], p.n)
    Rd = dense.rows_to_dense_R(rows, p.cf, p.n)
    scale = np.maximum(np.max(np.abs(Rd), axis=1, keepdims=True), 1e-300)
    assert np.max(np.abs(R - Rd) / scale) <= 1e-12


@pytest.mark.parametrize("case", range(len(CASES)))
def test_literal_algorithm1_with_aggregates(case):
    p = CASES[case](2)
    B = np.random.default_rng(case).uniform(0.5, 1.5, p.n)
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    _, o = _pats(p, B=B)
    R = dense.csr_to_dense_R(o["row_ptr"], o["col_idx"], o["val"], p.n)
    R1 = literal.algorithm1_R(A, p.cf, B, 2, k=1, agg=p.agg)
    assert np.max(np.abs(R1 - R)) <= 1e-12 * np.max(np.abs(R))
