"""GPU interpolation P = W(A) and the device CSR transpose.

Algorithm 1 (Section 3.1.3) builds interpolation from A and restriction from
A^T (Section 4.2 uses both for nonsymmetric problems); the library forms
P = (restriction of A^T)^T on the device (clair_build_P).  Checks:

* clair_transpose against scipy's transpose, entry by entry (exact: values
  are copied), square and rectangular, with empty rows and columns;
* clair_build_P against the oracle: P^T must equal the oracle's restriction
  of A^T (identical pattern, row error <= 1e-10, constraint residual
  <= 1e-12), both precisions, with and without a strength threshold;
* P injects the C-points and its constraint holds: P B_c = B on the covered
  F-points.
"""
import dataclasses

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2307_00229_amd import problems as P

from ._util import assert_matches_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_00229_amd import clair

    clair.load_library()


def _dev_csr(M):
    from paper_2307_00229_amd import clair

    M = sp.csr_matrix(M)
    M.sort_indices()
    return clair.CSR(torch.from_numpy(M.indptr.astype(np.int32)).cuda(),
                     torch.from_numpy(M.indices.astype(np.int32)).cuda(),
                     torch.from_numpy(M.data.astype(np.float64)).cuda(), n=M.shape[0])


def _transposed_problem(p):
    At = sp.csr_matrix(p.scipy().T)
    At.sort_indices()
    return dataclasses.replace(p, name=p.name + "_T", row_ptr=At.indptr.astype(np.int32),
                               col_idx=At.indices.astype(np.int32), val=At.data.astype(np.float64))


@pytest.mark.parametrize("case", range(4))
def test_transpose_matches_scipy(case):
    from paper_2307_00229_amd import clair

    rng = np.random.default_rng(case)
    if case == 0:
        M = P.cfg2()[0].scipy()
    elif case == 1:
        M = P.random_sparse(500, 0.01, 7).scipy()
    elif case == 2:  # rectangular, with empty rows and columns
        M = sp.random(300, 1000, density=0.003, random_state=3, format="csr")
        M.data = rng.standard_normal(M.nnz)
    else:  # the oracle's restriction (n_c x n)
        p = P.small_2d(40, stencil=9, eps=0.05, angle=1.0, k=3, ell=2)
        o = oracle.build_R_problem(p)
        M = sp.csr_matrix((o["val"], o["col_idx"], o["row_ptr"]), shape=(o["n_c"], p.n))
    M = sp.csr_matrix(M)
    M.sort_indices()
    print(f"[gpu] transpose case {case} shape {M.shape} nnz {M.nnz}", flush=True)
    rp, ci, va = clair.clair_transpose(_dev_csr(M), M.shape[1])
    T = sp.csr_matrix(M.T)
    T.sort_indices()
    assert np.array_equal(rp.cpu().numpy(), T.indptr)
    assert np.array_equal(ci.cpu().numpy(), T.indices)
    assert np.array_equal(va.cpu().numpy(), T.data)


def _check_P(p, precision, theta=0.0):
    from paper_2307_00229_amd import clair

    ctx = clair.Context()
    ctx.set_strength(theta)
    A = clair.CSR.from_problem(p)
    cf = torch.from_numpy(p.cf).cuda()
    B = None if p.B is None else torch.from_numpy(p.B).cuda()
    print(f"[gpu] build_P {p.name} precision={precision} theta={theta}", flush=True)
    (rp, ci, va), n_c, info, st = clair.clair_build_P(A, cf, B, p.ell, ctx=ctx, precision=precision)
    assert st == 0, info
    Pm = sp.csr_matrix((va.cpu().numpy(), ci.cpu().numpy(), rp.cpu().numpy()), shape=(p.n, n_c))
    Q = sp.csr_matrix(Pm.T)
    Q.sort_indices()
    pt = dataclasses.replace(_transposed_problem(p), theta=theta)
    g = dict(row_ptr=Q.indptr, col_idx=Q.indices, val=Q.data, n_c=n_c, nnz=Q.nnz)
    assert_matches_oracle(pt, g, oracle.build_R_problem(pt), info)
    # injection of the C-points
    C = np.nonzero(p.cf)[0]
    assert np.array_equal(Pm[C].toarray(), np.eye(n_c)) if n_c <= 2000 else True
    return Pm, C


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("case", range(3))
def test_build_P_matches_oracle(case, precision):
    p = [P.cfg2()[0], P.small_2d(120, stencil=9, eps=1e-3, angle=2.2, k=3, ell=2),
         P.random_sparse(600, 0.006, 9, ell=2)][case]
    Pm, C = _check_P(p, precision)
    if p.B is not None:
        # P B_c reproduces B on every F-point some column reaches
        F = np.nonzero(p.cf == 0)[0]
        covered = np.asarray((abs(Pm[F]) > 0).sum(axis=1)).ravel() > 0
        r = Pm @ p.B[C] - p.B
        assert np.max(np.abs(r[F][covered])) <= 1e-12 * max(1.0, np.max(np.abs(p.B)))


@pytest.mark.parametrize("theta", [0.25, 0.5])
def test_build_P_with_strength(theta):
    _check_P(P.small_2d(120, stencil=9, eps=1e-3, angle=2.2, k=3, ell=2), 0, theta)


def test_build_P_capacity_and_bad_arguments():
    from paper_2307_00229_amd import clair

    lib = clair.load_library()
    p = P.cfg1()
    A = clair.CSR.from_problem(p)
    cf = torch.from_numpy(p.cf).cuda()
    ctx = clair.Context()
    probe = clair.CsrOut()
    info = clair.Info()
    st = lib.clair_build_P(ctx.handle, A.c(), cf.data_ptr(), None, 1, probe, None, info)
    assert st == clair.CLAIR_ERR_CAPACITY and probe.n_rows == p.n and probe.nnz > 0
    st = lib.clair_build_P(ctx.handle, A.c(), cf.data_ptr(), None, 0, probe, None, info)
    assert st == clair.CLAIR_ERR_INVALID


def test_transpose_rejects_nnz_that_disagrees_with_row_ptr():
    # output buffers are sized from nnz and the kernels follow row_ptr: the
    # two must agree
    from paper_2307_00229_amd import clair

    M = sp.random(50, 40, density=0.1, random_state=5, format="csr")
    M.sort_indices()
    rp = torch.from_numpy(M.indptr.astype(np.int32)).cuda()
    ci = torch.from_numpy(np.concatenate([M.indices, [0, 1, 2]]).astype(np.int32)).cuda()
    va = torch.from_numpy(np.concatenate([M.data, [1.0, 2.0, 3.0]])).cuda()
    with pytest.raises(clair.ClairError) as ei:
        clair.clair_transpose(clair.CSR(rp, ci, va, n=50), 40)
    assert ei.value.status == clair.CLAIR_ERR_INVALID
