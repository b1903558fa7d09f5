"""GPU parity with a strength threshold theta on the pattern.

The paper's experiments grow the pattern from a classical strength matrix
with theta between 0.05 and 0.5 (Section 4).  Each case sets theta on the
context, builds R through the C ABI, and compares it with the oracle at the
same theta (oracle/clair_oracle.c, pinned by tests/test_oracle_strength.py):
identical pattern, row error <= 1e-10, constraint residual <= 1e-12.  Both
precisions, batches mixing matrices, graph replay, a plan, rows above 32
points (the workgroup search), and the 2048^2 recirculating workload at full
size.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2307_00229_amd import problems as P

from ._util import assert_matches_oracle, gpu_build, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_00229_amd import clair

    clair.load_library()


def _with_theta(ps, theta):
    return [dataclasses.replace(p, theta=theta) for p in ps]


def _run(ps, theta, precision=0):
    from paper_2307_00229_amd import clair

    ctx = clair.Context()
    ctx.set_strength(theta)
    assert ctx.get_strength() == theta
    print(f"[gpu] strength theta={theta} precision={precision} {[p.name for p in ps]}", flush=True)
    res, infos, st = gpu_build(ps, ctx=ctx, precision=precision)
    assert st == 0, (st, infos)
    for p, g, inf in zip(ps, res, infos):
        assert_matches_oracle(p, g, oracle.build_R_problem(p), inf)
    return res, infos


def _mixed_cases(ell=2):
    return [
        P.random_sparse(400, 0.01, 31, ell=ell),
        P.small_2d(48, stencil=9, eps=1e-3, angle=2.2, k=3, ell=ell),
        P.small_2d(64, stencil=5, eps=0.02, angle=0.4, ell=ell),
        P.small_3d(12, eps=0.05, b=(-1.0, 0.2, 0.7), ell=ell),
    ]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("theta", [0.05, 0.25, 0.5, 1.0])
def test_strength_parity_batched(theta, precision):
    ps = _with_theta(_mixed_cases(), theta)
    res, infos = _run(ps, theta, precision)
    # the threshold prunes the pattern: fewer entries than at theta = 0
    base = [oracle.build_R_problem(p, theta=0.0)["nnz"] for p in ps]
    assert sum(i["nnz"] for i in infos) < sum(base)


@pytest.mark.parametrize("theta", [0.3, 0.6])
def test_strength_large_blocks_workgroup_search(theta):
    # ell = 3 on a random pattern: rows of 33..106 (theta 0.3) and 33..58
    # (theta 0.6) points go through the workgroup search and solvers, which
    # apply the same test
    ps = _with_theta([P.random_sparse(600, 0.008, 41, ell=3, c_frac=0.2)], theta)
    o0 = oracle.build_R_problem(ps[0], theta=0.0)
    _, infos = _run(ps, theta)
    assert infos[0]["max_block"] > 32
    assert infos[0]["nnz"] < o0["nnz"]


def test_strength_recirculating_2048_full_size():
    ps = _with_theta([P.cfg3()], 0.25)
    _, infos = _run(ps, 0.25)
    assert infos[0]["n_c"] == 466489


def test_strength_graph_replay_and_plan():
    from paper_2307_00229_amd import clair

    theta = 0.25
    ps = _with_theta(_mixed_cases(), theta)
    As, cfs, Bs, ells = to_device(ps)
    ctx = clair.Context()
    ctx.set_strength(theta)
    eager, _, st = clair.clair_build_R_batched(As, cfs, Bs, ells, ctx=ctx)
    assert st == 0
    outs = [clair.ROut(o.n_c, o.nnz) for o in eager]
    s = torch.cuda.Stream()
    g = clair.Graph(ctx, As, cfs, Bs, ells, outs, stream=s)
    for _ in range(3):
        for o in outs:
            o.val.fill_(-7.0)
        torch.cuda.synchronize()
        g.launch(s)
        s.synchronize()
        st, infos = g.info()
        assert st == 0, infos
        clair.clair_build_R_batched(As, cfs, Bs, ells, ctx=ctx)  # eager work between replays
        for p, o, inf in zip(ps, outs, infos):
            rp, ci, va = o.trimmed()
            gres = dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(),
                        n_c=o.n_c, nnz=o.nnz)
            assert_matches_oracle(p, gres, oracle.build_R_problem(p), inf)
    g.close()
    # a plan created at this threshold keeps its pattern
    plan = clair.Plan(ctx, As, cfs, ells, outs)
    ctx.set_strength(0.0)  # later changes of the context do not touch the plan
    infos, st = plan.execute(As, Bs)
    assert st == 0
    for p, o, inf in zip(ps, outs, infos):
        rp, ci, va = o.trimmed()
        gres = dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(), n_c=o.n_c, nnz=o.nnz)
        assert_matches_oracle(p, gres, oracle.build_R_problem(p), inf)
    plan.close()


def test_strength_invalid_values_rejected():
    from paper_2307_00229_amd import clair

    ctx = clair.Context()
    ctx.set_strength(0.5)
    for bad in (-0.01, 1.01, float("nan")):
        with pytest.raises(clair.ClairError):
            ctx.set_strength(bad)
    assert ctx.get_strength() == 0.5


# --------------------------------------------- a strength matrix as input ---
def _csr_np(M):
    import scipy.sparse as sp

    M = sp.csr_matrix(M)
    M.sort_indices()
    return M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64)


def _dev_csr(rp, ci, va, n):
    from paper_2307_00229_amd import clair

    return clair.CSR(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), torch.from_numpy(va).cuda(), n=n)


def _random_graph(p, seed, keep=0.7, extra=0.01):
    """Part of A's couplings plus some that A does not have, as a 0/1 matrix."""
    import scipy.sparse as sp

    A = sp.csr_matrix((p.val, p.col_idx, p.row_ptr), shape=(p.n, p.n)).tocoo()
    rng = np.random.default_rng(seed)
    m = rng.random(A.nnz) < keep
    rows, cols = list(A.row[m]), list(A.col[m])
    k = int(extra * p.n * 4)
    rows += list(rng.integers(0, p.n, k))
    cols += list(rng.integers(0, p.n, k))
    S = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(p.n, p.n)).tocsr()
    S.data[:] = 1.0
    return _csr_np(S)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("ell", [2, 3])
def test_strength_matrix_batched(precision, ell):
    from paper_2307_00229_amd import clair

    ps = _mixed_cases(ell)[:3] if ell == 2 else [P.random_sparse(300, 0.01, 41, ell=3),
                                                 P.small_2d(40, stencil=9, eps=1e-2, angle=0.7, k=3, ell=3)]
    graphs = [_random_graph(p, 7 + k) for k, p in enumerate(ps)]
    ctx = clair.Context()
    ctx.set_graph([_dev_csr(*g, n=p.n) for g, p in zip(graphs, ps)])
    print(f"[gpu] strength matrix precision={precision} ell={ell} {[p.name for p in ps]}", flush=True)
    res, infos, st = gpu_build(ps, ctx=ctx, precision=precision)
    assert st == 0, (st, infos)
    for p, g, inf, gr in zip(ps, res, infos, graphs):
        o = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, strength=gr)
        assert_matches_oracle(p, g, o, inf)
    # the size query searches the same graph
    As, cfs, _, ells = to_device(ps)
    ncs, nzs = clair.clair_size_R(As, cfs, ells, ctx=ctx)
    assert list(nzs) == [i["nnz"] for i in infos]


def test_strength_matrix_of_the_threshold_rule_on_a_workload_matrix():
    # S holding exactly the strong couplings of A (|a_uv| >= theta max_w |a_wv|)
    # gives the build at that theta
    import scipy.sparse as sp

    from paper_2307_00229_amd import clair

    p = P.cfg2()[1]
    theta = 0.25
    A = sp.csr_matrix((p.val, p.col_idx, p.row_ptr), shape=(p.n, p.n)).tocoo()
    off = A.row != A.col
    colmax = np.zeros(p.n)
    np.maximum.at(colmax, A.col[off], np.abs(A.data[off]))
    strong = off & (np.abs(A.data) >= theta * colmax[A.col])
    S = _csr_np(sp.coo_matrix((np.ones(strong.sum()), (A.row[strong], A.col[strong])), shape=(p.n, p.n)))
    ctx = clair.Context()
    ctx.set_graph([_dev_csr(*S, n=p.n)])
    g, infos, st = gpu_build([p], ctx=ctx)
    assert st == 0, infos
    ctx2 = clair.Context()
    ctx2.set_strength(theta)
    h, infos2, st2 = gpu_build([p], ctx=ctx2)
    assert st2 == 0, infos2
    assert np.array_equal(g[0]["col_idx"], h[0]["col_idx"]) and np.array_equal(g[0]["row_ptr"], h[0]["row_ptr"])
    assert np.allclose(g[0]["val"], h[0]["val"], rtol=0, atol=1e-12 * np.abs(h[0]["val"]).max())


def test_strength_matrix_checks():
    from paper_2307_00229_amd import clair

    p = P.small_2d(20, stencil=5, eps=0.1, angle=0.5, ell=2)
    srp, sci, sva = _random_graph(p, 3)
    # a batch of a different size
    ctx = clair.Context()
    ctx.set_graph([_dev_csr(srp, sci, sva, p.n)])
    with pytest.raises(clair.ClairError) as ei:
        gpu_build([p, p], ctx=ctx)
    assert ei.value.status == clair.CLAIR_ERR_INVALID
    # an unsorted row is reported when validation is asked for
    bad = sci.copy()
    r = int(np.argmax(np.diff(srp) >= 2))
    bad[srp[r]], bad[srp[r] + 1] = bad[srp[r] + 1], bad[srp[r]]
    ctx.set_graph([_dev_csr(srp, bad, sva, p.n)])
    _, infos, st = gpu_build([p], ctx=ctx, validate=1, check=False)
    assert st == clair.CLAIR_ERR_INVALID
    # the P side would need a strength matrix of A^T
    ctx.set_graph([_dev_csr(srp, sci, sva, p.n)])
    A = clair.CSR.from_problem(p, "cuda")
    _, _, _, st = clair.clair_build_P(A, torch.from_numpy(p.cf).cuda(), None, p.ell, ctx=ctx, check=False)
    assert st == clair.CLAIR_ERR_UNSUPPORTED
    ctx.set_graph(None)
    _, infos, st = gpu_build([p], ctx=ctx)
    assert st == 0


def test_strength_matrix_graph_replay_and_plan():
    # graphs and plans created after clair_ctx_set_graph search the strength
    # matrices; replays and plan executes match the oracle on that graph
    from paper_2307_00229_amd import clair

    ps = _mixed_cases()[:3]
    graphs = [_random_graph(p, 21 + k) for k, p in enumerate(ps)]
    refs = [oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, strength=g) for p, g in zip(ps, graphs)]
    As, cfs, Bs, ells = to_device(ps)
    ctx = clair.Context()
    ctx.set_graph([_dev_csr(*g, n=p.n) for g, p in zip(graphs, ps)])
    eager, _, st = clair.clair_build_R_batched(As, cfs, Bs, ells, ctx=ctx)
    assert st == 0
    outs = [clair.ROut(o.n_c, o.nnz) for o in eager]
    s = torch.cuda.Stream()
    g = clair.Graph(ctx, As, cfs, Bs, ells, outs, stream=s)
    for _ in range(3):
        for o in outs:
            o.val.fill_(-7.0)
        torch.cuda.synchronize()
        g.launch(s)
        s.synchronize()
        st, infos = g.info()
        assert st == 0, infos
        clair.clair_build_R_batched(As, cfs, Bs, ells, ctx=ctx)  # eager work between replays
        for p, o, inf, ref in zip(ps, outs, infos, refs):
            rp, ci, va = o.trimmed()
            gres = dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(),
                        n_c=o.n_c, nnz=o.nnz)
            assert_matches_oracle(p, gres, ref, inf)
    g.close()
    plan = clair.Plan(ctx, As, cfs, ells, outs)
    infos, st = plan.execute(As, Bs)
    assert st == 0
    for p, o, inf, ref in zip(ps, outs, infos, refs):
        rp, ci, va = o.trimmed()
        gres = dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(), n_c=o.n_c, nnz=o.nnz)
        assert_matches_oracle(p, gres, ref, inf)
    plan.close()


def test_strength_matrix_in_the_approximate_and_kkt_builds():
    from oracle import kkt

    from paper_2307_00229_amd import clair

    from ._util import row_errors

    p = P.small_2d(30, stencil=9, eps=0.05, angle=1.0, k=3, ell=2)
    gr = _random_graph(p, 33)
    ctx = clair.Context()
    ctx.set_graph([_dev_csr(*gr, n=p.n)])
    A = clair.CSR.from_problem(p, "cuda")
    cf = torch.from_numpy(p.cf).cuda()
    B = torch.from_numpy(p.B).cuda()

    def as_dict(out, info):
        rp, ci, va = out
        return dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(), n_c=info["n_c"],
                    nnz=info["nnz"])

    out, info, _ = clair.clair_build_R_approx(A, cf, B, p.ell, 2, inverse=clair.CLAIR_INVERSE_ILU0, ctx=ctx)
    g = as_dict(out, info)
    o = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, 2, "ilu0", strength=gr)
    assert np.array_equal(g["col_idx"], o["col_idx"])
    assert row_errors(p, g, o)[0].max() <= 1e-10
    out, info, _ = clair.clair_build_R_kkt(A, cf, B, p.ell, ctx=ctx)
    g = as_dict(out, info)
    o = kkt.kkt_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, strength=gr)
    assert np.array_equal(g["col_idx"], o["col_idx"])
    assert row_errors(p, g, o)[0].max() <= 1e-10
