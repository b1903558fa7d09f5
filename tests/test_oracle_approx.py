"""Oracle pins for Algorithm 1 with the diagonal block inverse (CPU).

oracle.build_R_diag runs Algorithm 1's iteration with the local diagonal
inverse of every block (Section 3.1.2's approximate block inverses; the
diagonal one is the root-node-like variant of the footnote in the comparison
with root-node) on the exact build's pattern, column by column.  Pinned
against:
* the literal Algorithm 1 (oracle/literal.py: Q assembled entry by entry,
  pinv of Q Q^T, dense diagonal block inverses) for 0..4 iterations, with and
  without constraints;
* an exactness case: on a 5-point grid at distance 1 with C = (even, even),
  the four neighbours of a C-point are not coupled to each other, every block
  is diagonal, so the diagonal inverse is exact and one iteration gives the
  closed form; more iterations change nothing (Remark 2);
* the limit without constraints: the iteration is Jacobi on each local system,
  which converges on these row-dominant matrices to the exact l-AIR rows;
* feasibility: every iterate meets R^T B_c = B on the covered F-columns (the
  start is a feasible point and every update is projected);
* a zero diagonal on a pattern column is reported as singular.
"""
import numpy as np
import pytest

import oracle
from oracle import dense, literal
from paper_2307_00229_amd import problems as P

CASES = [
    lambda: P.small_2d(10, stencil=9, eps=0.05, angle=1.0, k=3, ell=2),
    lambda: P.small_2d(12, stencil=5, eps=0.1, angle=0.5, ell=2),
    lambda: P.small_3d(5, eps=0.05, b=(1.0, 0.3, -0.2), ell=2),
    lambda: P.random_sparse(50, 0.06, 5, ell=2),
]


def _dense_R(o, n):
    return dense.csr_to_dense_R(o["row_ptr"], o["col_idx"], o["val"], n)


@pytest.mark.parametrize("iters", [0, 1, 2, 4])
@pytest.mark.parametrize("constrained", [True, False])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_equals_literal_algorithm1(case, constrained, iters):
    p = CASES[case]()
    B = p.B if constrained else None
    got = oracle.build_R_diag(p.n, p.row_ptr, p.col_idx, p.val, p.cf, B, p.ell, iters)
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    Rl = literal.algorithm1_R(A, p.cf, B, p.ell, k=iters, inverse="diag")
    R = _dense_R(got, p.n)
    assert np.max(np.abs(Rl - R)) <= 1e-12 * max(1.0, np.max(np.abs(R)))


def test_diagonal_blocks_make_one_iteration_exact():
    p = P.cfg1()  # 32 x 32 5-point, distance 1, C = (even, even)
    exact = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)
    for iters in (1, 3):
        got = oracle.build_R_diag(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, iters)
        assert np.array_equal(got["col_idx"], exact["col_idx"])
        assert np.allclose(got["val"], exact["val"], rtol=0, atol=1e-14 * np.abs(exact["val"]).max())
    # zero iterations is not the closed form: the start is the minimum-norm fit
    got0 = oracle.build_R_diag(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, 0)
    assert np.abs(got0["val"] - exact["val"]).max() > 1e-3


@pytest.mark.parametrize("case", [1, 2, 3])
def test_unconstrained_limit_is_exact_lair(case):
    p = CASES[case]()
    exact = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell)
    got = oracle.build_R_diag(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell, 300)
    assert np.array_equal(got["col_idx"], exact["col_idx"])
    assert np.max(np.abs(got["val"] - exact["val"])) <= 1e-10 * np.abs(exact["val"]).max()
    # and the error falls with the iteration count
    errs = [np.abs(oracle.build_R_diag(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell, k)["val"]
                   - exact["val"]).max() for k in (1, 4, 16)]
    assert errs[0] > errs[1] > errs[2]


@pytest.mark.parametrize("iters", [0, 1, 3])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_every_iterate_meets_the_constraint(case, iters):
    p = CASES[case]()
    got = oracle.build_R_diag(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, iters)
    C = np.nonzero(p.cf)[0]
    rows = np.repeat(np.arange(got["n_c"]), np.diff(got["row_ptr"]))
    fm = got["col_idx"] != C[rows]
    terms = got["val"][fm] * p.B[C[rows[fm]]]
    S = np.zeros(p.n)
    T = np.zeros(p.n)
    np.add.at(S, got["col_idx"][fm], terms)
    np.add.at(T, got["col_idx"][fm], np.abs(terms))
    cov = np.zeros(p.n, bool)
    cov[got["col_idx"][fm]] = True
    res = np.abs(S[cov] - p.B[cov]) / (np.abs(p.B[cov]) + T[cov])
    assert res.max() <= 1e-13


def test_zero_diagonal_is_singular():
    p = P.small_2d(10, stencil=5, eps=0.1, angle=0.5, ell=2)
    va = p.val.copy()
    F = np.nonzero(p.cf == 0)[0]
    j = int(F[len(F) // 2])
    for e in range(p.row_ptr[j], p.row_ptr[j + 1]):
        if p.col_idx[e] == j:
            va[e] = 0.0
    with pytest.raises(oracle.OracleError):
        oracle.build_R_diag(p.n, p.row_ptr, p.col_idx, va, p.cf, p.B, p.ell, 1)


def _edge_problems():
    p0 = P.small_2d(12, ell=2)
    p0.cf = np.zeros(p0.n, np.int8)
    p1 = P.small_2d(12, ell=2)
    p1.cf = np.ones(p1.n, np.int8)
    iso = P.Problem("iso", 3, np.array([0, 2, 4, 6], np.int32), np.array([0, 1, 0, 1, 1, 2], np.int32),
                    np.array([2.0, -1.0, -1.0, 2.0, -1.0, 2.0]), np.array([1, 1, 0], np.int8), np.ones(3), 2)
    empty = P.Problem("empty", 0, np.array([0], np.int32), np.zeros(0, np.int32), np.zeros(0),
                      np.zeros(0, np.int8), np.zeros(0), 1)
    return [p0, p1, iso, empty]


@pytest.mark.parametrize("idx", range(4))
def test_degenerate_inputs(idx):
    # no C-points, all C-points, a C-point with no F-neighbour, n = 0
    p = _edge_problems()[idx]
    got = oracle.build_R_diag(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, 2)
    n_c = int((p.cf != 0).sum())
    assert got["n_c"] == n_c
    exact = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)
    assert np.array_equal(got["row_ptr"], exact["row_ptr"]) and np.array_equal(got["col_idx"], exact["col_idx"])
    assert got["n_uncovered"] == exact["n_uncovered"]
    if idx in (1, 2):  # every row is a bare injection
        C = np.nonzero(p.cf)[0]
        rows = np.repeat(np.arange(n_c), np.diff(got["row_ptr"]))
        assert np.all(got["val"][got["col_idx"] == C[rows]] == 1.0)
    if idx == 0:
        assert got["n_uncovered"] == p.n


# ---------------------------------------------------------------- ILU(0) ---
def _tridiag_1d(n=60, eps=0.1, b=1.0):
    """1D upwind advection-diffusion on n interior nodes, every third node C."""
    h = 1.0 / (n + 1)
    rp, ci, va = [0], [], []
    for r in range(n):
        row = []
        if r > 0:
            row.append((r - 1, -eps / h**2 - b / h))
        row.append((r, 2 * eps / h**2 + b / h))
        if r < n - 1:
            row.append((r + 1, -eps / h**2))
        for c_, v in row:
            ci.append(c_)
            va.append(v)
        rp.append(len(ci))
    cf = np.array([1 if r % 3 == 0 else 0 for r in range(n)], np.int8)
    return P.Problem("tridiag1d", n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va), cf,
                     np.ones(n), 2)


@pytest.mark.parametrize("seed", range(6))
def test_ilu0_factors_agree_with_the_block_on_its_pattern(seed):
    # the defining property of ILU(0): L U = K at every nonzero of K, with L
    # (unit lower) and U (upper) supported on K's pattern
    rng = np.random.default_rng(seed)
    s = 3 + seed * 3
    K = np.where(rng.random((s, s)) < 0.35, -rng.uniform(0.1, 1.0, (s, s)), 0.0)
    np.fill_diagonal(K, np.abs(K).sum(axis=1) + rng.uniform(0.5, 1.5, s))
    L, U = literal._ilu0(K)
    Pm = K != 0
    assert np.allclose((L @ U)[Pm], K[Pm], rtol=1e-13, atol=1e-13 * np.abs(K).max())
    assert np.all((np.tril(L, -1) != 0) <= Pm) and np.all((U != 0) <= Pm)
    assert np.allclose(np.diag(L), 1.0)


@pytest.mark.parametrize("iters", [0, 1, 3])
@pytest.mark.parametrize("constrained", [True, False])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_ilu0_equals_literal_algorithm1(case, constrained, iters):
    p = CASES[case]()
    B = p.B if constrained else None
    got = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, B, p.ell, iters, "ilu0")
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    Rl = literal.algorithm1_R(A, p.cf, B, p.ell, k=iters, inverse="ilu0")
    R = _dense_R(got, p.n)
    assert np.max(np.abs(Rl - R)) <= 1e-12 * max(1.0, np.max(np.abs(R)))


def test_ilu0_exact_on_tridiagonal_blocks():
    # 1D, distance 2, every third node C: each block is two uncoupled 2 x 2
    # pairs, which have no fill, so ILU(0) is the exact inverse and one
    # iteration gives the closed form; the diagonal inverse does not
    p = _tridiag_1d()
    exact = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)
    for iters in (1, 2):
        got = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, iters, "ilu0")
        assert np.array_equal(got["col_idx"], exact["col_idx"])
        assert np.allclose(got["val"], exact["val"], rtol=0, atol=1e-13 * np.abs(exact["val"]).max())
    diag = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, 1, "diag")
    assert np.abs(diag["val"] - exact["val"]).max() > 1e-3 * np.abs(exact["val"]).max()


@pytest.mark.parametrize("case", [1, 2, 3])
def test_ilu0_unconstrained_limit_is_exact_lair(case):
    # on these M-matrices ILU(0) is a convergent splitting of every block
    p = CASES[case]()
    exact = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell)
    got = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell, 100, "ilu0")
    assert np.max(np.abs(got["val"] - exact["val"])) <= 1e-10 * np.abs(exact["val"]).max()
    # and it gets there faster than the diagonal
    e_ilu = np.abs(oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell, 3, "ilu0")["val"]
                   - exact["val"]).max()
    e_dia = np.abs(oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell, 3, "diag")["val"]
                   - exact["val"]).max()
    assert e_ilu < e_dia


@pytest.mark.parametrize("case", range(len(CASES)))
def test_ilu0_iterates_meet_the_constraint(case):
    p = CASES[case]()
    got = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, 2, "ilu0")
    C = np.nonzero(p.cf)[0]
    rows = np.repeat(np.arange(got["n_c"]), np.diff(got["row_ptr"]))
    fm = got["col_idx"] != C[rows]
    terms = got["val"][fm] * p.B[C[rows[fm]]]
    S = np.zeros(p.n)
    T = np.zeros(p.n)
    np.add.at(S, got["col_idx"][fm], terms)
    np.add.at(T, got["col_idx"][fm], np.abs(terms))
    cov = np.zeros(p.n, bool)
    cov[got["col_idx"][fm]] = True
    assert (np.abs(S[cov] - p.B[cov]) / (np.abs(p.B[cov]) + T[cov])).max() <= 1e-13


# ----------------------------------------------------------------- GMRES ---
@pytest.mark.parametrize("krylov", [1, 2, 3])
@pytest.mark.parametrize("constrained", [True, False])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_gmres_equals_literal_algorithm1(case, constrained, krylov):
    # Arnoldi with Givens rotations (C oracle) against a least-squares fit over
    # an orthonormal basis of the Krylov space (literal)
    p = CASES[case]()
    B = p.B if constrained else None
    for iters in (1, 2):
        got = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, B, p.ell, iters, "gmres", krylov=krylov)
        A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
        Rl = literal.algorithm1_R(A, p.cf, B, p.ell, k=iters, inverse="gmres", krylov=krylov)
        R = _dense_R(got, p.n)
        assert np.max(np.abs(Rl - R)) <= 1e-10 * max(1.0, np.max(np.abs(R)))


def test_gmres_one_step_is_the_minimal_residual_multiple():
    # one GMRES step: u = alpha rho with alpha = (rho . K rho) / |K rho|^2
    p = CASES[1]()
    A = dense.to_dense(p.n, p.row_ptr, p.col_idx, p.val)
    got = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell, 1, "gmres", krylov=1)
    R = _dense_R(got, p.n)
    nb = dense.neighbourhoods(A, p.cf, p.ell)
    for r, c in enumerate(np.nonzero(p.cf)[0]):
        N = nb[c]
        if len(N) == 0:
            continue
        K = A[np.ix_(N, N)].T
        z0 = -A[c, N]
        rho = -A[c, N] - K @ z0
        Kr = K @ rho
        alpha = (rho @ Kr) / (Kr @ Kr) if np.any(Kr) else 0.0
        assert np.allclose(R[r, N], z0 + alpha * rho, rtol=0, atol=1e-12 * max(1.0, np.abs(R[r]).max()))


@pytest.mark.parametrize("case", range(len(CASES)))
def test_gmres_with_a_full_krylov_space_is_exact(case):
    # with as many steps as the block has points GMRES solves the block exactly,
    # so one iteration gives the closed form (Remark 2)
    p = CASES[case]()
    exact = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)
    got = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, 1, "gmres", krylov=64)
    assert np.array_equal(got["col_idx"], exact["col_idx"])
    assert np.max(np.abs(got["val"] - exact["val"])) <= 1e-10 * np.abs(exact["val"]).max()


@pytest.mark.parametrize("case", [1, 2, 3])
def test_gmres_unconstrained_limit_and_feasibility(case):
    p = CASES[case]()
    exact = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell)
    got = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell, 40, "gmres", krylov=2)
    assert np.max(np.abs(got["val"] - exact["val"])) <= 1e-10 * np.abs(exact["val"]).max()
    g = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, 2, "gmres", krylov=3)
    C = np.nonzero(p.cf)[0]
    rows = np.repeat(np.arange(g["n_c"]), np.diff(g["row_ptr"]))
    fm = g["col_idx"] != C[rows]
    terms = g["val"][fm] * p.B[C[rows[fm]]]
    S = np.zeros(p.n)
    T = np.zeros(p.n)
    np.add.at(S, g["col_idx"][fm], terms)
    np.add.at(T, g["col_idx"][fm], np.abs(terms))
    cov = np.zeros(p.n, bool)
    cov[g["col_idx"][fm]] = True
    assert (np.abs(S[cov] - p.B[cov]) / (np.abs(p.B[cov]) + T[cov])).max() <= 1e-13
