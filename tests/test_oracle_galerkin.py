"""Pins of the sparse-product reference used for the Galerkin operator (CPU).

``dense.product_reference`` (structural pattern of X Y, values, rounding
scale) is checked against dense NumPy products, including products that
cancel exactly (their column stays, with value 0), and R A P built from
oracle transfer operators against the dense triple product.
"""
import numpy as np
import scipy.sparse as sp

import oracle
from oracle import dense
from paper_2307_00229_amd import problems as P


def test_product_reference_equals_dense_product():
    rng = np.random.default_rng(3)
    for trial in range(5):
        X = sp.random(40, 55, density=0.08, random_state=trial, format="csr")
        Y = sp.random(55, 30, density=0.08, random_state=100 + trial, format="csr")
        X.data = rng.standard_normal(X.nnz)
        Y.data = rng.standard_normal(Y.nnz)
        C, S = dense.product_reference(X, Y)
        Xd, Yd = X.toarray(), Y.toarray()
        assert np.array_equal(S.toarray() > 0, (np.abs(Xd) @ np.abs(Yd)) > 0)
        assert np.allclose(C.toarray(), Xd @ Yd, rtol=0, atol=1e-14)
        assert np.array_equal(C.indptr, S.indptr) and np.array_equal(C.indices, S.indices)


def test_product_reference_keeps_cancelled_columns():
    X = sp.csr_matrix(np.array([[1.0, 1.0, 0.0]]))
    Y = sp.csr_matrix(np.array([[2.0, 1.0], [-2.0, 0.0], [5.0, 0.0]]))
    C, S = dense.product_reference(X, Y)
    assert C.indices.tolist() == [0, 1]
    assert C.data.tolist() == [0.0, 1.0]
    assert S.data.tolist() == [4.0, 1.0]


def test_galerkin_of_oracle_operators_equals_dense_triple_product():
    p = P.small_2d(14, stencil=9, eps=0.05, angle=1.2, k=3, ell=2)
    A = p.scipy()
    o = oracle.build_R_problem(p)
    R = sp.csr_matrix((o["val"], o["col_idx"], o["row_ptr"]), shape=(o["n_c"], p.n))
    At = sp.csr_matrix(A.T)
    At.sort_indices()
    q = oracle.build_R(p.n, At.indptr, At.indices, At.data, p.cf, p.B, p.ell)
    Pm = sp.csr_matrix((q["val"], q["col_idx"], q["row_ptr"]), shape=(q["n_c"], p.n)).T.tocsr()
    AP, _ = dense.product_reference(A, Pm)
    Ac, _ = dense.product_reference(R, AP)
    ref = R.toarray() @ A.toarray() @ Pm.toarray()
    assert np.allclose(Ac.toarray(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
