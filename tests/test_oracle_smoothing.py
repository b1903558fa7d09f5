"""Pins of the CFF-weighted-Jacobi smoothing of B (CPU).

Closed forms and invariants that the definition fixes:
* M diagonal: every sweep scales the points it touches by (1 - omega), so
  after k iterations C-entries carry (1 - omega)^k and F-entries
  (1 - omega)^(2k);
* a null vector of M is a fixed point (zero row sums: B = 1 for M = A;
  zero column sums: B = 1 for M = A^T);
* omega = 0 or zero iterations: B unchanged;
* linearity in B;
* a sweep leaves the points outside its subset alone, and for one point
  with one neighbour gives the hand value.
"""
import numpy as np
import scipy.sparse as sp

from oracle import smoothing as S
from paper_2307_00229_amd import problems as P


def test_diagonal_matrix_closed_form():
    rng = np.random.default_rng(0)
    n = 50
    A = sp.diags(rng.uniform(1.0, 3.0, n)).tocsr()
    cf = (rng.random(n) < 0.3).astype(np.int8)
    B = rng.standard_normal(n)
    om, k = 0.6, 4
    x = S.cff_jacobi(A, cf, B, k, om)
    want = np.where(cf != 0, B * (1 - om) ** k, B * (1 - om) ** (2 * k))
    assert np.allclose(x, want, rtol=1e-14, atol=0)


def test_null_vector_is_fixed():
    rng = np.random.default_rng(1)
    n = 80
    W = sp.random(n, n, density=0.05, random_state=2, format="lil")
    for i in range(n):  # a ring, so every row has a neighbour
        W[i, (i + 1) % n] = 1.0
    W = sp.csr_matrix(W)
    W.data = rng.uniform(0.1, 1.0, W.nnz)
    W.setdiag(0.0)
    W.eliminate_zeros()
    L = sp.csr_matrix(sp.diags(np.asarray(W.sum(axis=1)).ravel()) - W)  # zero row sums
    cf = (rng.random(n) < 0.25).astype(np.int8)
    one = np.ones(n)
    x = S.cff_jacobi(L, cf, one, 5, 0.7)
    assert np.allclose(x, 1.0, rtol=0, atol=1e-12)
    Lt = sp.csr_matrix(L.T)  # M = Lt^T = L for the transposed sweeps
    x2 = S.cff_jacobi(Lt, cf, one, 5, 0.7, transpose=True)
    assert np.allclose(x2, 1.0, rtol=0, atol=1e-12)
    # and B = 1 is not fixed for the transpose of a matrix without zero column sums
    x3 = S.cff_jacobi(L, cf, one, 5, 0.7, transpose=True)
    assert np.max(np.abs(x3 - 1.0)) > 1e-3


def test_identity_cases_and_linearity():
    p = P.small_2d(20, stencil=9, eps=0.05, angle=1.0, k=3, ell=2)
    A = p.scipy()
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(p.n), rng.standard_normal(p.n)
    assert np.array_equal(S.cff_jacobi(A, p.cf, u, 0, 0.7), u)
    assert np.array_equal(S.cff_jacobi(A, p.cf, u, 3, 0.0), u)
    for tr in (False, True):
        lhs = S.cff_jacobi(A, p.cf, 2.0 * u - 3.0 * v, 5, 0.7, tr)
        rhs = 2.0 * S.cff_jacobi(A, p.cf, u, 5, 0.7, tr) - 3.0 * S.cff_jacobi(A, p.cf, v, 5, 0.7, tr)
        assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def test_sweep_touches_only_its_subset_and_hand_value():
    # M = [[2, -1], [-4, 8]], x = (1, 1), sweep on point 0 with omega = 0.5:
    # (M x)_0 = 1, x_0 <- 1 - 0.5 * 1 / 2 = 0.75; x_1 unchanged
    M = sp.csr_matrix(np.array([[2.0, -1.0], [-4.0, 8.0]]))
    x = S.jacobi_subset(M, np.ones(2), np.array([True, False]), 0.5)
    assert x.tolist() == [0.75, 1.0]
    # the same on A^T: (M^T x)_0 = 2 - 4 = -2, x_0 <- 1 + 0.5 * 2 / 2 = 1.5
    xt = S.jacobi_subset(M.T, np.ones(2), np.array([True, False]), 0.5)
    assert xt.tolist() == [1.5, 1.0]
