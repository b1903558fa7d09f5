"""GPU normal-equations (KKT) minimiser (clair_build_R_kkt) against the oracle
(oracle.kkt.kkt_R, a direct sparse solve).

Section 3.1.1 states the constrained problem and its KKT system; Algorithm 1
projects in the Euclidean norm instead, and this entry point gives the exact
minimiser for comparison.  Checks: identical pattern and row error <= 1e-10
against the oracle on 2D / 3D / random nonsymmetric matrices and a 128^2
matrix of the workload's kind; equality with the Euclidean build where every
block is a multiple of I (5-point grid, distance 1); B = NULL gives the
unconstrained rows.
"""
import numpy as np
import pytest

from oracle import kkt
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
    lambda: P.cfg2(N=128)[0],
    lambda: P.cfg2(N=128)[2],
]


def _gpu_kkt(p, B):
    from paper_2307_00229_amd import clair

    A = clair.CSR.from_problem(p, "cuda")
    cf = torch.from_numpy(p.cf).cuda()
    Bt = None if B is None else torch.from_numpy(np.ascontiguousarray(B)).cuda()
    (rp, ci, va), info, st = clair.clair_build_R_kkt(A, cf, Bt, p.ell)
    torch.cuda.synchronize()
    return dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(), n_c=info["n_c"],
                nnz=info["nnz"]), info


@pytest.mark.parametrize("case", range(len(CASES)))
def test_matches_oracle(case):
    p = CASES[case]()
    g, info = _gpu_kkt(p, p.B)
    o = kkt.kkt_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)
    assert np.array_equal(g["row_ptr"], o["row_ptr"]) and np.array_equal(g["col_idx"], o["col_idx"])
    err, _, _ = row_errors(p, g, o)
    res, _ = constraint_residual(p, g)
    print(f"[gpu] kkt {p.name}: row error {err.max():.2e}, constraint {res:.2e}, "
          f"CG steps {info['refine_iters_max']}", flush=True)
    assert err.max() <= 1e-10
    assert res <= 1e-12


def test_equals_euclidean_where_blocks_are_multiples_of_identity():
    p = P.cfg1()
    g, _ = _gpu_kkt(p, p.B)
    ex, infos, st = gpu_build([p])
    assert st == 0, infos
    err, _, _ = row_errors(p, g, ex[0])
    assert err.max() <= 1e-10, err.max()


def test_without_B_is_the_unconstrained_build():
    import dataclasses

    p = CASES[1]()
    g, _ = _gpu_kkt(p, None)
    ex, infos, st = gpu_build([dataclasses.replace(p, B=None)])
    assert st == 0, infos
    assert np.array_equal(g["val"], ex[0]["val"])


@pytest.mark.parametrize("idx", range(4))
def test_degenerate_inputs(idx):
    # no C-points, all C-points, a C-point with no F-neighbour, n = 0
    from .test_oracle_approx import _edge_problems

    p = _edge_problems()[idx]
    print(f"[gpu] kkt degenerate {p.name} n={p.n}", flush=True)
    g, _ = _gpu_kkt(p, p.B)
    o = kkt.kkt_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)
    assert g["n_c"] == o["n_c"]
    assert np.array_equal(g["row_ptr"], o["row_ptr"]) and np.array_equal(g["col_idx"], o["col_idx"])
    assert np.allclose(g["val"], o["val"], rtol=0, atol=1e-14)
