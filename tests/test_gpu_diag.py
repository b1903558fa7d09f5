"""GPU Algorithm 1 with the diagonal block inverse (clair_build_R_diag)
against the oracle (oracle.build_R_diag).

Section 3.1.2 allows approximate block inverses; the local diagonal inverse is
the root-node-like variant of the footnote in the comparison with root-node.
Checks:
* pattern identical and row error <= 1e-10 against the oracle for 0..4
  iterations, with and without B, on 2D / 3D / random nonsymmetric matrices,
  with a strength threshold, and on a 512 x 512 workload matrix;
* on a 5-point grid at distance 1 every block is diagonal, so one iteration
  equals the exact build (clair_build_R) to 1e-10;
* every iterate meets the constraint (<= 1e-12 of its terms), n_uncovered as
  the oracle's;
* a zero diagonal on a pattern column is CLAIR_ERR_SINGULAR with the smallest
  C-point whose row meets it.
"""
import numpy as np
import pytest

import oracle
from paper_2307_00229_amd import problems as P

from ._util import constraint_residual, gpu_build, row_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_00229_amd import clair

    clair.load_library()


CASES = [
    lambda: P.small_2d(12, stencil=9, eps=0.05, angle=1.0, k=3, ell=2),
    lambda: P.small_2d(40, stencil=5, eps=0.1, angle=0.5, ell=2),
    lambda: P.small_3d(9, eps=0.05, b=(1.0, 0.3, -0.2), ell=2),
    lambda: P.random_sparse(400, 0.01, 5, ell=2),
    lambda: P.cfg1(),
]


def _gpu_diag(p, B, iters, theta=0.0):
    from paper_2307_00229_amd import clair

    ctx = clair.Context()
    if theta:
        ctx.set_strength(theta)
    A = clair.CSR.from_problem(p, "cuda")
    cf = torch.from_numpy(p.cf).cuda()
    Bt = None if B is None else torch.from_numpy(np.ascontiguousarray(B)).cuda()
    (rp, ci, va), info, st = clair.clair_build_R_diag(A, cf, Bt, p.ell, iters, ctx=ctx)
    torch.cuda.synchronize()
    return dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(), n_c=info["n_c"],
                nnz=info["nnz"]), info


def _compare(p, B, iters, theta=0.0):
    g, info = _gpu_diag(p, B, iters, theta)
    o = oracle.build_R_diag(p.n, p.row_ptr, p.col_idx, p.val, p.cf, B, p.ell, iters, theta=theta)
    assert np.array_equal(g["row_ptr"], o["row_ptr"]) and np.array_equal(g["col_idx"], o["col_idx"])
    err, _, _ = row_errors(p, g, o)
    print(f"[gpu] diag {p.name} B={'yes' if B is not None else 'no'} iters={iters} theta={theta}: "
          f"row error {err.max():.2e}", flush=True)
    assert err.max() <= 1e-10
    if B is not None:
        assert info["n_uncovered"] == o["n_uncovered"]
    return g, o


@pytest.mark.parametrize("iters", [0, 1, 2, 4])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_matches_oracle_with_B(case, iters):
    p = CASES[case]()
    g, _ = _compare(p, p.B, iters)
    res, _ = constraint_residual(p, g)
    assert res <= 1e-12, res


@pytest.mark.parametrize("iters", [0, 3])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_matches_oracle_without_B(case, iters):
    p = CASES[case]()
    _compare(p, None, iters)


@pytest.mark.parametrize("case", [0, 2])
def test_strength_threshold(case):
    p = CASES[case]()
    _compare(p, p.B, 2, theta=0.25)


def test_one_iteration_exact_on_diagonal_blocks():
    p = P.cfg1()
    g, _ = _gpu_diag(p, p.B, 1)
    ex, infos, st = gpu_build([p])
    assert st == 0, infos
    assert np.array_equal(g["col_idx"], ex[0]["col_idx"])
    err, _, _ = row_errors(p, g, ex[0])
    assert err.max() <= 1e-10, err.max()


def test_workload_matrix():
    p = P.cfg2()[1]
    _compare(p, p.B, 3)


def test_zero_diagonal_is_singular():
    from paper_2307_00229_amd import clair

    p = P.small_2d(10, stencil=5, eps=0.1, angle=0.5, ell=2)
    va = p.val.copy()
    F = np.nonzero(p.cf == 0)[0]
    j = int(F[len(F) // 2])
    for e in range(p.row_ptr[j], p.row_ptr[j + 1]):
        if p.col_idx[e] == j:
            va[e] = 0.0
    q = P.Problem(p.name, p.n, p.row_ptr, p.col_idx, va, p.cf, p.B, p.ell)
    pat = oracle.build_R(q.n, q.row_ptr, q.col_idx, q.val, q.cf, None, q.ell, allow_singular=True)
    C = np.nonzero(q.cf)[0]
    rows = np.repeat(np.arange(pat["n_c"]), np.diff(pat["row_ptr"]))
    expect = int(C[rows[pat["col_idx"] == j]].min())
    A = clair.CSR.from_problem(q, "cuda")
    (_, info, st) = clair.clair_build_R_diag(A, torch.from_numpy(q.cf).cuda(), torch.from_numpy(q.B).cuda(), q.ell,
                                            1, check=False)
    assert st == clair.CLAIR_ERR_SINGULAR
    assert info["first_bad_row"] == expect


@pytest.mark.parametrize("idx", range(4))
def test_degenerate_inputs(idx):
    # no C-points, all C-points, a C-point with no F-neighbour, n = 0
    from .test_oracle_approx import _edge_problems

    p = _edge_problems()[idx]
    print(f"[gpu] diag degenerate {p.name} n={p.n} n_c={int((p.cf != 0).sum())}", flush=True)
    g, info = _gpu_diag(p, p.B, 2)
    o = oracle.build_R_diag(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, 2)
    assert g["n_c"] == o["n_c"]
    assert np.array_equal(g["row_ptr"], o["row_ptr"]) and np.array_equal(g["col_idx"], o["col_idx"])
    assert np.allclose(g["val"], o["val"], rtol=0, atol=1e-14)
    assert info["n_uncovered"] == o["n_uncovered"]


# ---------------------------------------------------------------- ILU(0) ---
def _gpu_approx(p, B, iters, inverse, theta=0.0, check=True, krylov=0):
    from paper_2307_00229_amd import clair

    ctx = clair.Context()
    if theta:
        ctx.set_strength(theta)
    A = clair.CSR.from_problem(p, "cuda")
    cf = torch.from_numpy(p.cf).cuda()
    Bt = None if B is None else torch.from_numpy(np.ascontiguousarray(B)).cuda()
    out, info, st = clair.clair_build_R_approx(A, cf, Bt, p.ell, iters, inverse=inverse, krylov=krylov, ctx=ctx,
                                               check=check)
    torch.cuda.synchronize()
    if out is None or st:
        return None, info, st
    rp, ci, va = out
    return dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(), n_c=info["n_c"],
                nnz=info["nnz"]), info, st


def _compare_ilu(p, B, iters, theta=0.0):
    from paper_2307_00229_amd import clair

    g, info, _ = _gpu_approx(p, B, iters, clair.CLAIR_INVERSE_ILU0, theta)
    o = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, B, p.ell, iters, "ilu0", theta=theta)
    assert np.array_equal(g["row_ptr"], o["row_ptr"]) and np.array_equal(g["col_idx"], o["col_idx"])
    err, _, _ = row_errors(p, g, o)
    print(f"[gpu] ilu0 {p.name} B={'yes' if B is not None else 'no'} iters={iters} theta={theta}: "
          f"row error {err.max():.2e}", flush=True)
    assert err.max() <= 1e-10
    if B is not None:
        assert info["n_uncovered"] == o["n_uncovered"]
        res, _ = constraint_residual(p, g)
        assert res <= 1e-12, res
    return g, o


@pytest.mark.parametrize("iters", [0, 1, 3])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_ilu0_matches_oracle(case, iters):
    p = CASES[case]()
    _compare_ilu(p, p.B, iters)
    _compare_ilu(p, None, iters)


def test_ilu0_strength_and_workload_matrix():
    _compare_ilu(CASES[0](), CASES[0]().B, 2, theta=0.25)
    p = P.cfg2()[0]
    _compare_ilu(p, p.B, 2)


def test_ilu0_one_iteration_exact_on_fill_free_blocks():
    from .test_oracle_approx import _tridiag_1d

    p = _tridiag_1d()
    from paper_2307_00229_amd import clair

    g, _, _ = _gpu_approx(p, p.B, 1, clair.CLAIR_INVERSE_ILU0)
    ex, infos, st = gpu_build([p])
    assert st == 0, infos
    err, _, _ = row_errors(p, g, ex[0])
    assert err.max() <= 1e-10, err.max()


def test_ilu0_zero_pivot_is_singular():
    from paper_2307_00229_amd import clair

    p = P.small_2d(10, stencil=5, eps=0.1, angle=0.5, ell=2)
    va = p.val.copy()
    F = np.nonzero(p.cf == 0)[0]
    j = int(F[0])  # the first F-point: its diagonal is the first pivot of every block holding it first
    for e in range(p.row_ptr[j], p.row_ptr[j + 1]):
        if p.col_idx[e] == j:
            va[e] = 0.0
    q = P.Problem(p.name, p.n, p.row_ptr, p.col_idx, va, p.cf, p.B, p.ell)
    with pytest.raises(oracle.OracleError) as exc:
        oracle.build_R_approx(q.n, q.row_ptr, q.col_idx, q.val, q.cf, q.B, q.ell, 1, "ilu0")
    expect = int(str(exc.value).split("bad_row=")[1])
    _, info, st = _gpu_approx(q, q.B, 1, clair.CLAIR_INVERSE_ILU0, check=False)
    assert st == clair.CLAIR_ERR_SINGULAR
    assert info["first_bad_row"] == expect


# ----------------------------------------------------------------- GMRES ---
def _compare_gmres(p, B, iters, krylov, theta=0.0):
    from paper_2307_00229_amd import clair

    g, info, _ = _gpu_approx(p, B, iters, clair.CLAIR_INVERSE_GMRES, theta, krylov=krylov)
    o = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, B, p.ell, iters, "gmres", theta=theta,
                              krylov=krylov)
    assert np.array_equal(g["row_ptr"], o["row_ptr"]) and np.array_equal(g["col_idx"], o["col_idx"])
    err, _, _ = row_errors(p, g, o)
    print(f"[gpu] gmres({krylov}) {p.name} B={'yes' if B is not None else 'no'} iters={iters}: "
          f"row error {err.max():.2e}", flush=True)
    assert err.max() <= 1e-10
    if B is not None:
        assert info["n_uncovered"] == o["n_uncovered"]
        res, _ = constraint_residual(p, g)
        assert res <= 1e-12, res
    return g


@pytest.mark.parametrize("krylov", [1, 3])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_gmres_matches_oracle(case, krylov):
    p = CASES[case]()
    for iters in (1, 2):
        _compare_gmres(p, p.B, iters, krylov)
        _compare_gmres(p, None, iters, krylov)


def test_gmres_workload_matrix_and_strength():
    p = P.cfg2()[0]
    _compare_gmres(p, p.B, 2, 3)
    _compare_gmres(CASES[2](), CASES[2]().B, 2, 2, theta=0.25)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_gmres_full_krylov_space_is_exact(case):
    # every block of these matrices has at most 32 points
    from paper_2307_00229_amd import clair

    p = CASES[case]()
    g, _, _ = _gpu_approx(p, p.B, 1, clair.CLAIR_INVERSE_GMRES, krylov=32)
    ex, infos, st = gpu_build([p])
    assert st == 0, infos
    err, _, _ = row_errors(p, g, ex[0])
    print(f"[gpu] gmres(32) {p.name} vs exact build: row error {err.max():.2e}", flush=True)
    assert err.max() <= 1e-10, err.max()


def test_gmres_bad_krylov_rejected():
    from paper_2307_00229_amd import clair

    p = CASES[1]()
    for m in (0, 33):
        _, _, st = _gpu_approx(p, p.B, 1, clair.CLAIR_INVERSE_GMRES, krylov=m, check=False)
        assert st == clair.CLAIR_ERR_INVALID
