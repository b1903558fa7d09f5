"""GPU k > 1 constraint vectors (clair_project_constraints) against the oracle.

With k constraint vectors, Algorithm 1's Q holds k rows per F-point and Q Q^T
is block diagonal with k x k blocks (Section 3.1): each F-column j is
projected on its own, z_ij -= B_i^T pinv(G_j) r_j.  The device pass runs on an
R built without constraints; the oracle (oracle.project_constraints) runs on
the oracle's unconstrained R.  Checks:

* k = 1: the projected GPU R equals the GPU build with B and the oracle's
  constrained closed form (row error <= 1e-10);
* k = 2, 3, 4 (registers) and 6, 8 (LDS): every entry against the oracle, with the error allowed to grow
  with the conditioning of the column's Gram matrix (the projection's own
  amplification of the unconstrained rows' 1e-10 difference);
* the constraints hold on the GPU result for every full-rank F-column, and
  n_uncovered equals the oracle's;
* a 512 x 512 workload matrix (262144 unknowns) at k = 4;
* index errors and a row count other than the number of C-points are
  rejected, an R with no F-entries is left as it is, and two calls give the
  same bits (every column is summed in ascending row order).
"""
import numpy as np
import pytest

import oracle
from paper_2307_00229_amd import problems as P

from ._util import gpu_build, row_errors

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
    lambda: P.random_sparse(400, 0.01, 5, ell=2, B=None),
    lambda: P.cfg1(),
]


def _Bk(p, k, seed):
    rng = np.random.default_rng(seed)
    B = rng.uniform(0.5, 1.5, (p.n, k))
    if k > 1:
        B[:, 1] = np.linspace(-1.0, 1.0, p.n) + 0.1 * B[:, 1]
    return B


def _unconstrained(p):
    import dataclasses

    q = dataclasses.replace(p, B=None)
    res, infos, st = gpu_build([q])
    assert st == 0, infos
    return res[0]


def _project_gpu(p, g, B):
    from paper_2307_00229_amd import clair

    R = (torch.from_numpy(g["row_ptr"]).cuda(), torch.from_numpy(g["col_idx"]).cuda(),
         torch.from_numpy(g["val"]).cuda())
    unc = clair.clair_project_constraints(R, p.n, torch.from_numpy(p.cf).cuda(),
                                          torch.from_numpy(np.ascontiguousarray(B)).cuda())
    torch.cuda.synchronize()
    out = dict(g)
    out["val"] = R[2].cpu().numpy()
    out["n_uncovered"] = unc
    return out


def _gram(p, o, B):
    C = np.nonzero(p.cf)[0]
    rows = np.repeat(np.arange(o["n_c"]), np.diff(o["row_ptr"]))
    fm = o["col_idx"] != C[rows]
    Bi = B[C[rows[fm]]]
    k = B.shape[1]
    G = np.zeros((p.n, k, k))
    np.add.at(G, o["col_idx"][fm], Bi[:, :, None] * Bi[:, None, :])
    return G, fm, rows


def _cond_kept(G, rcond=1e-12):
    """Per column: largest over smallest kept eigenvalue of G_j (1 when empty)."""
    w = np.linalg.eigvalsh(G)
    wmax = np.abs(w).max(axis=1)
    kept = np.where(np.abs(w) > rcond * wmax[:, None], np.abs(w), np.inf)
    wmin = kept.min(axis=1)
    return np.where(np.isfinite(wmin) & (wmax > 0), wmax / np.where(np.isfinite(wmin), wmin, 1.0), 1.0)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_k1_equals_constrained_build(case):
    p = CASES[case]()
    B = _Bk(p, 1, case)
    g = _project_gpu(p, _unconstrained(p), B)
    pb = P.Problem(p.name, p.n, p.row_ptr, p.col_idx, p.val, p.cf, B[:, 0].copy(), p.ell)
    direct, infos, st = gpu_build([pb])
    assert st == 0, infos
    o = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, B[:, 0], p.ell)
    assert np.array_equal(g["col_idx"], o["col_idx"])
    err, _, _ = row_errors(pb, g, o)
    err_d, _, _ = row_errors(pb, g, direct[0])
    print(f"[gpu] k=1 {p.name}: vs oracle {err.max():.2e}, vs direct {err_d.max():.2e}", flush=True)
    assert err.max() <= 1e-10 and err_d.max() <= 1e-10
    assert g["n_uncovered"] == o["n_uncovered"]


@pytest.mark.parametrize("k", [2, 3, 4, 6, 8])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_matches_oracle(case, k):
    p = CASES[case]()
    B = _Bk(p, k, 40 + case)
    g = _project_gpu(p, _unconstrained(p), B)
    ou = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell)
    o = oracle.project_constraints(ou, p.cf, B)
    assert np.array_equal(g["col_idx"], o["col_idx"]) and np.array_equal(g["row_ptr"], o["row_ptr"])
    assert g["n_uncovered"] == o["n_uncovered"]
    G, fm, rows = _gram(p, o, B)
    cond = _cond_kept(G)
    scale = np.zeros(o["n_c"])
    np.maximum.at(scale, rows[fm], np.abs(o["val"][fm]))
    scale = np.maximum(scale, np.abs(ou["val"]).max() * 1e-3)
    bound = 1e-10 * scale[rows[fm]] * cond[o["col_idx"][fm]]
    d = np.abs(g["val"][fm] - o["val"][fm])
    print(f"[gpu] k={k} {p.name}: max err/bound {np.max(d / bound):.2e}, max cond {cond.max():.1e}", flush=True)
    assert np.all(d <= bound)
    # C-entries are untouched
    assert np.array_equal(g["val"][~fm], o["val"][~fm])
    # the constraints on full-rank columns
    C = np.nonzero(p.cf)[0]
    S = np.zeros((p.n, k))
    A = np.zeros((p.n, k))
    terms = g["val"][fm][:, None] * B[C[rows[fm]]]
    np.add.at(S, g["col_idx"][fm], terms)
    np.add.at(A, g["col_idx"][fm], np.abs(terms))
    w = np.linalg.eigvalsh(G)
    full = (w.min(axis=1) > 1e-8 * np.abs(w).max(axis=1)) & (p.cf == 0)
    if not full.any():
        # e.g. distance 1 on a 5-point grid: at most 2 rows reach a column,
        # fewer than k = 3 vectors; every column is then a least-squares fit
        rows_per_col = np.bincount(g["col_idx"][fm], minlength=p.n)
        assert rows_per_col.max() < k
        return
    res = np.abs(S[full] - B[full]) / (np.abs(B[full]) + A[full] + 1e-300)
    assert np.all(res <= 1e-13 * cond[full][:, None]), res.max()


def test_workload_matrix_k4():
    p = P.cfg2()[0]
    B = _Bk(p, 4, 99)
    g = _project_gpu(p, _unconstrained(p), B)
    o = oracle.project_constraints(oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell), p.cf, B)
    G, fm, rows = _gram(p, o, B)
    cond = _cond_kept(G)
    scale = np.zeros(o["n_c"])
    np.maximum.at(scale, rows[fm], np.abs(o["val"][fm]))
    d = np.abs(g["val"][fm] - o["val"][fm]) / (1e-10 * scale[rows[fm]] * cond[o["col_idx"][fm]])
    print(f"[gpu] k=4 {p.name}: max err/bound {d.max():.2e}, uncovered {g['n_uncovered']}", flush=True)
    assert d.max() <= 1.0
    assert g["n_uncovered"] == o["n_uncovered"]


def test_rejects_bad_index_and_arguments():
    from paper_2307_00229_amd import clair

    p = CASES[0]()
    g = _unconstrained(p)
    ci = g["col_idx"].copy()
    ci[len(ci) // 2] = p.n + 5  # outside [0, n): reported, no access made
    R = (torch.from_numpy(g["row_ptr"]).cuda(), torch.from_numpy(ci).cuda(), torch.from_numpy(g["val"]).cuda())
    cf = torch.from_numpy(p.cf).cuda()
    B = torch.ones(p.n, 2, dtype=torch.float64, device="cuda")
    with pytest.raises(clair.ClairError):
        clair.clair_project_constraints(R, p.n, cf, B)
    R = (torch.from_numpy(g["row_ptr"]).cuda(), torch.from_numpy(g["col_idx"]).cuda(),
         torch.from_numpy(g["val"]).cuda())
    with pytest.raises(clair.ClairError):  # k = 9
        clair.clair_project_constraints(R, p.n, cf, torch.ones(p.n, 9, dtype=torch.float64, device="cuda"))
    # one row fewer than C-points
    n_c = g["n_c"]
    Rs = (R[0][:n_c].contiguous(), R[1][: int(g["row_ptr"][n_c - 1])].contiguous(),
          R[2][: int(g["row_ptr"][n_c - 1])].contiguous())
    with pytest.raises(clair.ClairError):
        clair.clair_project_constraints(Rs, p.n, cf, B)


def test_deterministic():
    p = CASES[1]()
    B = _Bk(p, 3, 5)
    g = _unconstrained(p)
    a = _project_gpu(p, g, B)
    b = _project_gpu(p, g, B)
    assert np.array_equal(a["val"], b["val"])


def test_all_c_points_leaves_r_unchanged():
    from paper_2307_00229_amd import clair

    n = 50
    rp = torch.arange(n + 1, dtype=torch.int32, device="cuda")
    ci = torch.arange(n, dtype=torch.int32, device="cuda")
    va = torch.ones(n, dtype=torch.float64, device="cuda")
    cf = torch.ones(n, dtype=torch.int8, device="cuda")
    unc = clair.clair_project_constraints((rp, ci, va), n, cf, torch.rand(n, 3, dtype=torch.float64, device="cuda"))
    assert unc == 0
    assert torch.equal(va, torch.ones_like(va))


@pytest.mark.parametrize("idx", [0, 2, 3])
def test_degenerate_inputs(idx):
    # no C-points (every F-point uncovered), a C-point with no F-neighbour, n = 0
    from .test_oracle_approx import _edge_problems

    p = _edge_problems()[idx]
    print(f"[gpu] constraints degenerate {p.name} n={p.n}", flush=True)
    B = _Bk(p, 2, 7) if p.n else np.zeros((0, 2))
    g = _project_gpu(p, _unconstrained(p), B)
    o = oracle.project_constraints(oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, None, p.ell), p.cf, B)
    assert g["n_uncovered"] == o["n_uncovered"]
    assert np.allclose(g["val"], o["val"], rtol=0, atol=1e-14)


def test_rejects_nnz_that_disagrees_with_row_ptr():
    from paper_2307_00229_amd import clair

    p = CASES[0]()
    g = _unconstrained(p)
    R = (torch.from_numpy(g["row_ptr"]).cuda(),
         torch.from_numpy(np.concatenate([g["col_idx"], [0]]).astype(np.int32)).cuda(),
         torch.from_numpy(np.concatenate([g["val"], [0.0]])).cuda())
    with pytest.raises(clair.ClairError) as ei:
        clair.clair_project_constraints(R, p.n, torch.from_numpy(p.cf).cuda(),
                                        torch.ones(p.n, 2, dtype=torch.float64, device="cuda"))
    assert ei.value.status == clair.CLAIR_ERR_INVALID
