"""GPU smoothing of the constraint vector against the oracle.

clair_smooth_B (CFF-weighted Jacobi on A or A^T, Section 4) against
oracle/smoothing.py (pinned in tests/test_oracle_smoothing.py), entry by
entry within 1e-13 of the largest entry (products are fused on the GPU, so
the last bits differ); then R built on the GPU with the GPU-smoothed B
against the oracle's R with the oracle-smoothed B (the paper's setting:
B = 1 pre-smoothed with 5 iterations, weight 1 / rho(D^{-1} A)).
"""
import dataclasses

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import smoothing as S
from paper_2307_00229_amd import problems as P

from . import _vcycle as V
from ._util import assert_matches_oracle, gpu_build

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_00229_amd import clair

    clair.load_library()


CASES = [
    lambda: P.cfg2()[1],
    lambda: P.small_2d(200, stencil=9, eps=1e-3, angle=2.2, k=3, ell=2),
    lambda: P.small_3d(24, eps=1e-2, b=(1.0, 0.5, 0.25), ell=2),
    lambda: P.random_sparse(3000, 0.002, 4, ell=2),
]


def _omega(A):
    return 1.0 / V.arnoldi_rho(sp.diags(1.0 / A.diagonal()) @ A)


@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_smoothing_matches_oracle(case, transpose):
    from paper_2307_00229_amd import clair

    p = CASES[case]()
    A = p.scipy()
    om = _omega(A)
    B0 = np.random.default_rng(case).uniform(0.5, 1.5, p.n)
    ref = S.cff_jacobi(A, p.cf, B0, 5, om, transpose)
    print(f"[gpu] smooth {p.name} transpose={transpose} omega={om:.4f}", flush=True)
    got = clair.clair_smooth_B(clair.CSR.from_problem(p), torch.from_numpy(p.cf).cuda(),
                               torch.from_numpy(B0).cuda(), 5, om, transpose=transpose).cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.max(np.abs(ref - B0)) > 1e-6  # the sweeps did something


def test_restriction_with_smoothed_constraint():
    from paper_2307_00229_amd import clair

    p = P.cfg2()[2]
    A = p.scipy()
    om = _omega(A)
    ones = np.ones(p.n)
    Bref = S.cff_jacobi(A, p.cf, ones, 5, om, transpose=True)
    Bdev = clair.clair_smooth_B(clair.CSR.from_problem(p), torch.from_numpy(p.cf).cuda(),
                                torch.from_numpy(ones).cuda(), 5, om, transpose=True)
    # the GPU setup with the GPU-smoothed vector against the oracle with the oracle's
    q = dataclasses.replace(p, B=Bdev.cpu().numpy())
    res, infos, st = gpu_build([q])
    assert st == 0
    assert_matches_oracle(dataclasses.replace(p, B=Bref), res[0], oracle.build_R_problem(dataclasses.replace(p, B=Bref)),
                          infos[0])


def test_in_place_and_errors():
    from paper_2307_00229_amd import clair

    p = CASES[0]()
    A = clair.CSR.from_problem(p)
    cf = torch.from_numpy(p.cf).cuda()
    B = torch.ones(p.n, dtype=torch.float64, device="cuda")
    ref = S.cff_jacobi(p.scipy(), p.cf, np.ones(p.n), 2, 0.6)
    clair.clair_smooth_B(A, cf, B, 2, 0.6, out=B)  # in place
    assert np.max(np.abs(B.cpu().numpy() - ref)) <= 1e-13
    # a zero diagonal on a swept point
    M = sp.csr_matrix(np.array([[0.0, -1.0], [-1.0, 2.0]]))
    Z = clair.CSR(torch.from_numpy(M.indptr.astype(np.int32)).cuda(), torch.from_numpy(M.indices.astype(np.int32)).cuda(),
                  torch.from_numpy(M.data).cuda(), n=2)
    with pytest.raises(clair.ClairError) as ei:
        clair.clair_smooth_B(Z, torch.tensor([1, 0], dtype=torch.int8, device="cuda"),
                             torch.ones(2, dtype=torch.float64, device="cuda"), 1, 0.5)
    assert ei.value.status == clair.CLAIR_ERR_SINGULAR
