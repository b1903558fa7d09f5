"""Oracle pins for the strength-filtered pattern (CPU only).

Algorithm 1 (Section 3.1.3) takes the pattern of W from the classical strength
matrix S of the matrix it is applied to; R is Algorithm 1 on A^T, and the
paper's experiments use thresholds theta = 0.05 to 0.5 (Section 4).  The C
oracle walks A's rows from each C-point and tests each step u -> v against the
largest off-diagonal magnitude of column v (the transposition worked out in
its header).  These tests pin that walk against:

* a hand-worked four-point example where a row-based reading would give a
  different pattern;
* ``dense.neighbourhoods``: S of A^T formed literally (row maxima of A^T) and
  the expansion S^{m-1} T by boolean matrix products;
* theta = 0 equal to the plain stored-nonzero graph of A, written out here;
* monotonicity in theta, and the theta = 1, ell = 1 pattern written out;
* unconstrained rows equal to dense solves, and the literal Algorithm 1 equal
  to the closed form, on strength-filtered patterns.
"""
import numpy as np
import pytest

import oracle
from oracle import dense, literal
from paper_2307_00229_amd import problems as P


def _csr(A):
    n = A.shape[0]
    rp, ci, va = [0], [], []
    for r in range(n):
        cols = np.nonzero(A[r])[0]
        ci.extend(cols.tolist())
        va.extend(A[r, cols].tolist())
        rp.append(len(ci))
    return np.asarray(rp, np.int32), np.asarray(ci, np.int32), np.asarray(va, np.float64)


def _patterns(p, theta, B=None):
    o = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, B, p.ell, theta=theta)
    C = np.nonzero(p.cf)[0]
    pats = {}
    for r, i in enumerate(C):
        cols = o["col_idx"][o["row_ptr"][r]:o["row_ptr"][r + 1]]
        pats[int(i)] = [int(c) for c in cols if c != i]
    return pats, o


def test_hand_example_uses_column_maxima():
    # points 0 (C), 1, 2, 3 (F); ell = 1, theta = 0.5
    #   a_01 = -1, a_02 = -0.1, a_31 = -5
    # column maxima (off-diagonal): cmax_1 = 5, cmax_2 = 0.1
    #   0 -> 1: |a_01| = 1   >= 0.5 * 5   = 2.5  fails
    #   0 -> 2: |a_02| = 0.1 >= 0.5 * 0.1 = 0.05 holds
    # so N(0) = {2}.  (Measuring against row 0's own maximum, 1, would keep 1
    # and drop 2 instead.)
    A = np.array([[4.0, -1.0, -0.1, 0.0],
                  [0.0, 4.0, 0.0, 0.0],
                  [0.0, 0.0, 4.0, 0.0],
                  [0.0, -5.0, 0.0, 9.0]])
    rp, ci, va = _csr(A)
    p = P.Problem("hand4", 4, rp, ci, va, np.array([1, 0, 0, 0], np.int8), None, 1)
    pats, _ = _patterns(p, 0.5)
    assert pats == {0: [2]}
    assert dense.neighbourhoods(A, p.cf, 1, 0.5) [0].tolist() == [2]
    # theta = 0: both neighbours
    pats0, _ = _patterns(p, 0.0)
    assert pats0 == {0: [1, 2]}


CASES = [
    lambda ell: P.random_sparse(40, 0.08, 21, ell=ell, B=None),
    lambda ell: P.random_sparse(36, 0.12, 22, ell=ell, nonsym_pattern=False, B=None),
    lambda ell: P.small_2d(9, stencil=9, eps=1e-3, angle=2.2, k=3, ell=ell),
    lambda ell: P.small_2d(10, stencil=5, eps=0.02, angle=0.4, ell=ell),
    lambda ell: P.small_3d(5, eps=0.05, b=(-1.0, 0.2, 0.7), ell=ell),
]


@pytest.mark.parametrize("theta", [0.05, 0.25, 0.5, 1.0])
@pytest.mark.parametrize("ell", [1, 2, 3])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_pattern_equals_literal_strength_expansion(case, ell, theta):
    p = CASES[case](ell)
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    pats, _ = _patterns(p, theta)
    nb = dense.neighbourhoods(A, p.cf, ell, theta)
    assert pats == {i: v.tolist() for i, v in nb.items()}


@pytest.mark.parametrize("case", range(len(CASES)))
def test_theta_zero_is_the_stored_nonzero_graph(case):
    p = CASES[case](2)
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    n = p.n
    adj = (A != 0) & ~np.eye(n, dtype=bool)  # u -> v when a_uv != 0
    F = p.cf == 0
    pats, _ = _patterns(p, 0.0)
    for i in np.nonzero(p.cf)[0]:
        reach = adj[i] & F
        reach = reach | ((reach.astype(np.int64) @ adj.astype(np.int64)) > 0) & F
        assert pats[int(i)] == np.nonzero(reach)[0].tolist()
    nb = dense.neighbourhoods(A, p.cf, 2, 0.0)
    assert pats == {i: v.tolist() for i, v in nb.items()}


@pytest.mark.parametrize("case", range(len(CASES)))
def test_patterns_shrink_as_theta_grows(case):
    p = CASES[case](3)
    prev = None
    for theta in [0.0, 0.1, 0.3, 0.6, 1.0]:
        pats, _ = _patterns(p, theta)
        if prev is not None:
            for i, v in pats.items():
                assert set(v) <= set(prev[i])
        prev = pats


@pytest.mark.parametrize("case", range(len(CASES)))
def test_theta_one_distance_one_keeps_the_column_maxima(case):
    p = CASES[case](1)
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    off = np.abs(A) * (1 - np.eye(p.n))
    cmax = off.max(axis=0)
    pats, _ = _patterns(p, 1.0)
    for i in np.nonzero(p.cf)[0]:
        want = [v for v in range(p.n) if v != i and p.cf[v] == 0 and A[i, v] != 0 and abs(A[i, v]) >= cmax[v]]
        assert pats[int(i)] == want


@pytest.mark.parametrize("theta", [0.05, 0.5])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_strength_rows_equal_dense_solves(case, theta):
    p = CASES[case](2)
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    rows = dense.lair_rows(A, p.cf, 2, theta)
    _, o = _patterns(p, theta)
    R = dense.csr_to_dense_R(o["row_ptr"], o["col_idx"], o["val"], p.n)
    Rd = dense.rows_to_dense_R(rows, p.cf, p.n)
    scale = np.maximum(np.max(np.abs(Rd), axis=1, keepdims=True), 1e-300)
    assert np.max(np.abs(R - Rd) / scale) <= 1e-12


@pytest.mark.parametrize("case", [0, 2, 4])
def test_literal_algorithm1_with_strength_matches_closed_form(case):
    p = CASES[case](2)
    rng = np.random.default_rng(100 + case)
    B = rng.uniform(0.5, 1.5, p.n)
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    _, o = _patterns(p, 0.25, B=B)
    R = dense.csr_to_dense_R(o["row_ptr"], o["col_idx"], o["val"], p.n)
    R1 = literal.algorithm1_R(A, p.cf, B, 2, k=1, theta=0.25)
    assert np.max(np.abs(R1 - R)) <= 1e-12 * np.max(np.abs(R))


def test_invalid_theta_rejected():
    p = CASES[0](2)
    for bad in (-0.1, 1.5, float("nan")):
        with pytest.raises(oracle.OracleError):
            oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, 2, theta=bad)


# --------------------------------------------- a strength matrix as input ---
def _csr(M):
    import scipy.sparse as sp

    M = sp.csr_matrix(M)
    M.sort_indices()
    return M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64)


def test_strength_matrix_equal_to_A_changes_nothing():
    p = P.small_2d(14, stencil=9, eps=0.05, angle=1.0, k=3, ell=2)
    a = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)
    b = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, strength=(p.row_ptr, p.col_idx, p.val))
    assert np.array_equal(a["col_idx"], b["col_idx"]) and np.array_equal(a["val"], b["val"])


@pytest.mark.parametrize("seed", range(3))
def test_strength_matrix_is_the_search_graph(seed):
    # a random graph that drops some of A's couplings and adds others: the
    # pattern is dense reachability on S (F-interiors), the rows still solve
    # the systems of A on that pattern
    import scipy.sparse as sp

    p = P.random_sparse(60, 0.06, 10 + seed, ell=2)
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    rng = np.random.default_rng(seed)
    S = np.where((A != 0) & (rng.random(A.shape) < 0.7), 1.0, 0.0)
    S += np.where(rng.random(A.shape) < 0.01, 1.0, 0.0)
    np.fill_diagonal(S, 1.0)
    srp, sci, sva = _csr(S)
    got = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell, strength=(srp, sci, sva))
    nb = dense.neighbourhoods(S, p.cf, p.ell)
    C = np.nonzero(p.cf)[0]
    for r, i in enumerate(C):
        e = np.arange(got["row_ptr"][r], got["row_ptr"][r + 1])
        cols = got["col_idx"][e]
        N = np.asarray(nb[int(i)], int)
        assert np.array_equal(cols[cols != i], N)
        if len(N):
            z = np.linalg.solve(A[np.ix_(N, N)].T, -A[i, N])
            assert np.allclose(got["val"][e][cols != i], z, rtol=0, atol=1e-12 * max(1.0, np.abs(z).max()))


# ------------------------------------- the literal S^{ell-1} T pattern ---
@pytest.mark.parametrize("theta", [0.0, 0.25])
def test_literal_pattern_agrees_up_to_distance_2_and_not_beyond(theta):
    # Algorithm 1 expands T = [S_fc, I] by S^{ell-1}, which lets C-points be
    # interior vertices; the searches here keep F-points only.  Both give the
    # same pattern for ell <= 2 (every workload), and from ell = 3 on the
    # literal one can be larger
    cases = [P.small_2d(12, stencil=9, eps=0.05, angle=1.0, k=3), P.small_2d(14, stencil=5, eps=0.1, angle=0.5),
             P.small_3d(5, eps=0.05, b=(1.0, 0.3, -0.2)), P.random_sparse(60, 0.06, 5)]
    larger = 0
    for p in cases:
        A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
        for ell in (1, 2, 3):
            ours = dense.neighbourhoods(A, p.cf, ell, theta)
            lit = dense.neighbourhoods_literal(A, p.cf, ell, theta)
            for c in ours:
                assert set(ours[c]) <= set(lit[c])
                if ell <= 2:
                    assert np.array_equal(ours[c], lit[c]), (p.name, ell, c)
                else:
                    larger += len(lit[c]) > len(ours[c])
    assert larger > 0


@pytest.mark.parametrize("theta", [0.0, 0.25])
def test_literal_search_equals_the_boolean_products(theta):
    # the C oracle's literal search (C-points as interior vertices) against
    # pattern((S^{ell-1} T)|_F) formed by boolean matrix products, ell = 1..4
    cases = [P.small_2d(12, stencil=9, eps=0.05, angle=1.0, k=3), P.small_2d(14, stencil=5, eps=0.1, angle=0.5),
             P.small_3d(5, eps=0.05, b=(1.0, 0.3, -0.2)), P.random_sparse(60, 0.06, 5)]
    for p in cases:
        A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
        for ell in (1, 2, 3, 4):
            lit = dense.neighbourhoods_literal(A, p.cf, ell, theta)
            o = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, ell, theta=theta, literal=True,
                               allow_singular=True)
            C = np.nonzero(p.cf)[0]
            for r, c in enumerate(C):
                cols = o["col_idx"][o["row_ptr"][r]:o["row_ptr"][r + 1]]
                assert np.array_equal(cols[cols != c], lit[int(c)]), (p.name, ell, int(c))
            if ell <= 2:
                d = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, ell, theta=theta)
                assert np.array_equal(d["col_idx"], o["col_idx"]) and np.array_equal(d["val"], o["val"])


def _lit_cols(p_n, rp, ci, va, cf, ell, theta):
    o = oracle.build_R(p_n, rp, ci, va, cf, None, ell, theta=theta, literal=True, allow_singular=True)
    C = np.nonzero(cf)[0]
    out = {}
    for r, c in enumerate(C):
        cols = o["col_idx"][o["row_ptr"][r]:o["row_ptr"][r + 1]]
        out[int(c)] = cols[cols != c]
    return out


def test_literal_search_c_point_without_f_neighbours():
    # T = [S_fc, I] puts the C-point itself in T's column, so the first step
    # of S^{ell-1} expands it even when it has no (strong) F-neighbour: its
    # C-neighbours become interior vertices.  1D Laplacian, n = 6,
    # C = {0, 1, 4}: C-point 0 reaches 2 through 1 at distance 3 (by hand:
    # T's column 0 is {0}; S steps give {0, 1}, then {0, 1, 2}; F part {2})
    n = 6
    A = np.diag(np.full(n, 2.0)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
    cf = np.array([1, 1, 0, 0, 1, 0], dtype=np.int8)
    rp, ci, va = _csr(A)
    for ell in (1, 2, 3, 4):
        got = _lit_cols(n, rp, ci, va, cf, ell, 0.0)
        want = dense.neighbourhoods_literal(A, cf, ell)
        for c in want:
            assert np.array_equal(got[c], want[c]), (ell, c)
    assert _lit_cols(n, rp, ci, va, cf, 3, 0.0)[0].tolist() == [2]
    assert _lit_cols(n, rp, ci, va, cf, 2, 0.0)[0].tolist() == []
    # a C-point whose only F-neighbour is weak at theta = 0.5: C-point 0 has
    # F-neighbour 1 (|a_01| = 0.1 against column 1's largest off-diagonal 1)
    # and C-neighbour 2 (strong); through 2 it reaches F-point 3 at distance 3
    B = np.zeros((6, 6))
    for u, v, a in [(0, 1, 0.1), (0, 2, 1.0), (1, 0, 1.0), (1, 3, 1.0), (2, 0, 1.0), (2, 3, 1.0), (3, 1, 1.0),
                    (3, 2, 1.0), (3, 4, 1.0), (4, 3, 1.0), (4, 5, 1.0), (5, 4, 1.0)]:
        B[u, v] = -a
    np.fill_diagonal(B, 4.0)
    cf2 = np.array([1, 0, 1, 0, 0, 1], dtype=np.int8)
    rp, ci, va = _csr(B)
    for ell in (1, 2, 3, 4):
        got = _lit_cols(6, rp, ci, va, cf2, ell, 0.5)
        want = dense.neighbourhoods_literal(B, cf2, ell, 0.5)
        for c in want:
            assert np.array_equal(got[c], want[c]), (ell, c)
    assert _lit_cols(6, rp, ci, va, cf2, 3, 0.5)[0].tolist() == [3]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_literal_search_dense_c_points(seed):
    # many C-points, so that some have no F-neighbour or only weak ones: the
    # literal search against the boolean products, ell = 1..4
    rng = np.random.default_rng(100 + seed)
    p = P.random_sparse(50, 0.08, 20 + seed, ell=2)
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    cf = (rng.random(p.n) < 0.55).astype(np.int8)
    lacking = 0
    for theta in (0.0, 0.3):
        S = dense.strength_transposed(A, theta)
        for c in np.nonzero(cf)[0]:
            lacking += not np.any(S[:, c] & (cf == 0))
        for ell in (1, 2, 3, 4):
            got = _lit_cols(p.n, p.row_ptr, p.col_idx, p.val, cf, ell, theta)
            want = dense.neighbourhoods_literal(A, cf, ell, theta)
            for c in want:
                assert np.array_equal(got[c], want[c]), (theta, ell, c)
    assert lacking > 0
