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


def _read_cff_cases():
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "cff_jacobi_hand.txt")
    cases, cur = [], None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, _, rest = line.partition(" ")
        if key == "case":
            cur = {"name": rest}
            cases.append(cur)
        elif key == "A":
            cur["A"] = np.array([[float(v) for v in r.split()] for r in rest.split(";")])
        elif key in ("cf",):
            cur[key] = np.array([int(v) for v in rest.split()], dtype=np.int8)
        elif key in ("B", "x"):
            cur[key] = np.array([float(v) for v in rest.split()])
        elif key in ("iterations", "transpose"):
            cur[key] = int(rest)
        else:
            cur[key] = float(rest)
    return cases


def test_cff_order_hand_example():
    """Hand-worked CFF iterations on non-diagonal 3x3 matrices (every value a
    dyadic fraction, so exact in FP64): the sweep order C, F, F of Section 4's
    smoother is pinned, and the orders F, F, C and F, C, F miss the values."""
    cases = _read_cff_cases()
    assert [c["name"] for c in cases] == ["sym", "ns_T", "sym2"]
    for c in cases:
        A = sp.csr_matrix(c["A"])
        x = S.cff_jacobi(A, c["cf"], c["B"], c["iterations"], c["omega"], bool(c["transpose"]))
        assert x.tolist() == c["x"].tolist(), c["name"]
        # the same iteration with the sweeps reordered differs from the hand values
        M = sp.csr_matrix(A.T if c["transpose"] else A)
        Cm = c["cf"] != 0
        for order in ((~Cm, ~Cm, Cm), (~Cm, Cm, ~Cm)):
            y = c["B"].copy()
            for _ in range(c["iterations"]):
                for mask in order:
                    y = S.jacobi_subset(M, y, mask, c["omega"])
            assert y.tolist() != c["x"].tolist(), c["name"]
