"""GPU sparse products and the Galerkin coarse operator A_c = R A P.

clair_spgemm and clair_galerkin against ``dense.product_reference`` (the
structural pattern of the product and its values, pinned in
tests/test_oracle_galerkin.py): identical pattern, and every entry within
1e-13 of the sum of its terms' magnitudes (the summation order differs).
Then a whole hierarchy on the device -- R by clair_build_R, P by
clair_build_P, A_c by clair_galerkin on every level -- against the
hierarchy built from the oracle: coarse operators within 1e-10 and the same
V-cycle convergence factor to 3 digits (Section 4).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import dense
from paper_2307_00229_amd import problems as P

from . import _vcycle as V
from ._util import gpu_build

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_00229_amd import clair

    clair.load_library()


def _dev(M):
    from paper_2307_00229_amd import clair

    M = sp.csr_matrix(M)
    M.sort_indices()
    return clair.CSR(torch.from_numpy(M.indptr.astype(np.int32)).cuda(),
                     torch.from_numpy(M.indices.astype(np.int32)).cuda(),
                     torch.from_numpy(M.data.astype(np.float64)).cuda(), n=M.shape[0])


def _host(t, shape):
    rp, ci, va = (x.cpu().numpy() for x in t)
    return sp.csr_matrix((va, ci, rp), shape=shape)


def _assert_product(G, X, Y):
    C, S = dense.product_reference(X, Y)
    assert np.array_equal(G.indptr, C.indptr)
    assert np.array_equal(G.indices, C.indices)
    assert np.all(np.abs(G.data - C.data) <= 1e-13 * S.data + 1e-300)


@pytest.mark.parametrize("case", range(4))
def test_spgemm_matches_reference(case):
    from paper_2307_00229_amd import clair

    rng = np.random.default_rng(case)
    if case == 0:
        X = P.cfg2()[0].scipy()
        Y = X
    elif case == 1:  # rectangular, empty rows and columns
        X = sp.random(700, 900, density=0.004, random_state=5, format="csr")
        Y = sp.random(900, 400, density=0.01, random_state=6, format="csr")
        X.data, Y.data = rng.standard_normal(X.nnz), rng.standard_normal(Y.nnz)
    elif case == 2:  # cancelling products keep their column
        X = sp.csr_matrix(np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 0.0], [0.0, 3.0, 1.0]]))
        Y = sp.csr_matrix(np.array([[2.0, 1.0], [-2.0, 0.0], [5.0, 0.0]]))
    else:  # rows of a few hundred columns
        X = sp.random(200, 3000, density=0.006, random_state=7, format="csr")
        Y = sp.random(3000, 3000, density=0.004, random_state=8, format="csr")
        X.data, Y.data = rng.standard_normal(X.nnz), rng.standard_normal(Y.nnz)
    X, Y = sp.csr_matrix(X), sp.csr_matrix(Y)
    widest = int((abs(X) @ abs(Y) > 0).sum(axis=1).max())
    print(f"[gpu] spgemm case {case} {X.shape} x {Y.shape} widest row {widest}", flush=True)
    assert widest <= 1536
    G = _host(clair.clair_spgemm(_dev(X), X.shape[1], _dev(Y), Y.shape[1]), (X.shape[0], Y.shape[1]))
    _assert_product(G, X, Y)


def test_spgemm_rows_above_the_bound_and_bad_shapes():
    from paper_2307_00229_amd import clair

    rng = np.random.default_rng(9)
    X = sp.random(50, 8000, density=0.04, random_state=10, format="csr")
    Y = sp.random(8000, 8000, density=0.01, random_state=11, format="csr")
    X.data, Y.data = rng.standard_normal(X.nnz), rng.standard_normal(Y.nnz)
    X, Y = sp.csr_matrix(X), sp.csr_matrix(Y)
    assert int((abs(X) @ abs(Y) > 0).sum(axis=1).max()) > 1536
    with pytest.raises(clair.ClairError) as ei:
        clair.clair_spgemm(_dev(X), X.shape[1], _dev(Y), Y.shape[1])
    assert ei.value.status == clair.CLAIR_ERR_UNSUPPORTED
    with pytest.raises(clair.ClairError) as ei:  # inner dimensions differ
        clair.clair_spgemm(_dev(X), X.shape[1] + 1, _dev(Y), Y.shape[1])
    assert ei.value.status == clair.CLAIR_ERR_INVALID


def _oracle_RP(p):
    A = p.scipy()
    o = oracle.build_R_problem(p)
    R = sp.csr_matrix((o["val"], o["col_idx"], o["row_ptr"]), shape=(o["n_c"], p.n))
    At = sp.csr_matrix(A.T)
    At.sort_indices()
    q = oracle.build_R(p.n, At.indptr, At.indices, At.data, p.cf, p.B, p.ell)
    Pm = sp.csr_matrix(sp.csr_matrix((q["val"], q["col_idx"], q["row_ptr"]), shape=(q["n_c"], p.n)).T)
    Pm.sort_indices()
    return A, R, Pm


@pytest.mark.parametrize("case", range(3))
def test_galerkin_matches_reference(case):
    from paper_2307_00229_amd import clair

    p = [P.cfg2()[1], P.small_2d(150, stencil=9, eps=1e-3, angle=2.2, k=3, ell=2),
         P.small_3d(20, eps=1e-2, b=(1.0, 0.5, 0.25), ell=2)][case]
    A, R, Pm = _oracle_RP(p)
    print(f"[gpu] galerkin {p.name}", flush=True)
    G = _host(clair.clair_galerkin(_dev(R), _dev(A), _dev(Pm), R.shape[0]), (R.shape[0], R.shape[0]))
    AP, _ = dense.product_reference(A, Pm)
    Ac, S = dense.product_reference(R, AP)
    # the triple product's terms: |R| |A| |P|
    _, S3 = dense.product_reference(abs(R), abs(A) @ abs(Pm))
    assert np.array_equal(G.indptr, Ac.indptr) and np.array_equal(G.indices, Ac.indices)
    assert np.all(np.abs(G.data - Ac.data) <= 1e-13 * S3.data + 1e-300)


def _gpu_level_ops():
    from paper_2307_00229_amd import clair

    ctx = clair.Context()

    def build_R(parts, cf, B, ell):
        n, rp, ci, va = parts
        prob = P.Problem("level", n, rp, ci, va, cf.astype(np.int8), B, ell)
        res, infos, st = gpu_build([prob], ctx=ctx)
        assert st == 0, infos
        g = res[0]
        return sp.csr_matrix((g["val"], g["col_idx"], g["row_ptr"]), shape=(g["n_c"], n))

    def build_P(parts, cf, B, ell):
        n, rp, ci, va = parts
        A = clair.CSR(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), torch.from_numpy(va).cuda(), n=n)
        (prp, pci, pva), n_c, info, st = clair.clair_build_P(A, torch.from_numpy(cf.astype(np.int8)).cuda(),
                                                             torch.from_numpy(B).cuda(), ell, ctx=ctx)
        return sp.csr_matrix((pva.cpu().numpy(), pci.cpu().numpy(), prp.cpu().numpy()), shape=(n, n_c))

    def galerkin(R, A, Pm):
        return _host(clair.clair_galerkin(_dev(R), _dev(A), _dev(Pm), R.shape[0], ctx=ctx),
                     (R.shape[0], R.shape[0]))

    return build_R, build_P, galerkin


@pytest.mark.parametrize("idx", [0, 2])
def test_device_hierarchy_matches_oracle_hierarchy(idx):
    p = P.cfg2()[idx]
    A = p.scipy()
    bR, bP, gal = _gpu_level_ops()
    print(f"[gpu] device hierarchy {p.name}", flush=True)
    orc = V.build_hierarchy(A, (512, 512), 2, p.ell, V.oracle_builder(), max_levels=4)
    gpu = V.build_hierarchy(A, (512, 512), 2, p.ell, bR, max_levels=4, build_P=bP, galerkin=gal)
    assert len(orc) == len(gpu)
    for lo, lg in zip(orc[1:], gpu[1:]):
        d = abs(lo.A - lg.A).max()
        assert d <= 1e-10 * abs(lo.A).max(), d
    g_o, g_g = V.convergence_factor(orc), V.convergence_factor(gpu)
    print(f"[gpu] gamma oracle={g_o:.6f} device={g_g:.6f}", flush=True)
    assert abs(g_g - g_o) <= 5e-4 * g_o, (g_g, g_o)
