"""GPU: the literal S^{ell-1} T pattern (clair_ctx_set_literal_pattern).

Algorithm 1 expands T = [S_fc, I] by S^{ell-1}; taken literally, C-points can
be interior vertices of a walk from distance 3 on (the oracle's literal
search is pinned against boolean matrix products in
tests/test_oracle_strength.py).  The per-row FP64 form searches literally
for any ell: pattern identical and row error <= 1e-10 against the oracle at
ell = 3, where the literal patterns are larger; the size query agrees; the
approximate-inverse build (which uses that form's pattern) too.  The mixed
path gives the same bits as the default reading at ell <= 2 (where the
readings agree) and matches the oracle's literal pattern at ell = 3 and 4,
through its register search, its workgroup search and its workgroup solver.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2307_00229_amd import problems as P

from ._util import assert_matches_oracle, gpu_build, row_errors, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_00229_amd import clair

    clair.load_library()


def _cases(ell):
    return [P.small_2d(40, stencil=5, eps=0.1, angle=0.5, ell=ell),
            P.small_3d(9, eps=0.05, b=(1.0, 0.3, -0.2), ell=ell),
            P.random_sparse(300, 0.01, 5, ell=ell)]


def _ctx():
    from paper_2307_00229_amd import clair

    ctx = clair.Context()
    ctx.set_literal_pattern(True)
    return ctx


def test_fp64_form_searches_literally_at_distance_3():
    from paper_2307_00229_amd import clair

    ps = _cases(3)
    ctx = _ctx()
    print(f"[gpu] literal pattern, FP64 form, ell=3 {[p.name for p in ps]}", flush=True)
    res, infos, st = gpu_build(ps, ctx=ctx, precision=clair.CLAIR_PREC_FP64)
    assert st == 0, infos
    larger = 0
    for p, g, inf in zip(ps, res, infos):
        o = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, literal=True)
        assert_matches_oracle(p, g, o, inf)
        larger += o["nnz"] > oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)["nnz"]
    assert larger > 0
    As, cfs, _, ells = to_device(ps)
    ncs, nzs = clair.clair_size_R(As, cfs, ells, ctx=ctx)
    assert list(nzs) == [i["nnz"] for i in infos]


def test_mixed_path_agrees_at_distance_2():
    ps = _cases(2)
    a, _, st = gpu_build(ps, ctx=_ctx())
    assert st == 0
    b, _, st = gpu_build(ps)
    assert st == 0
    for x, y in zip(a, b):  # the same pattern, and the same bits (every sum has a fixed order)
        assert np.array_equal(x["row_ptr"], y["row_ptr"]) and np.array_equal(x["col_idx"], y["col_idx"])
        assert np.array_equal(x["val"], y["val"])


@pytest.mark.parametrize("ell", [3, 4])
def test_mixed_path_searches_literally(ell):
    # the register search with C-points as interior vertices, the workgroup
    # search for rows that pass more than 32 vertices (the random pattern and
    # ell = 4), and the workgroup solver's own search for blocks above 32
    from paper_2307_00229_amd import clair

    ps = _cases(ell) + [P.small_2d(48, stencil=9, eps=1e-2, angle=0.7, k=3, ell=ell)]
    ctx = _ctx()
    print(f"[gpu] literal pattern, mixed form, ell={ell} {[p.name for p in ps]}", flush=True)
    res, infos, st = gpu_build(ps, ctx=ctx)
    assert st == 0, infos
    larger = 0
    for p, g, inf in zip(ps, res, infos):
        o = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, literal=True)
        assert_matches_oracle(p, g, o, inf)
        larger += o["nnz"] > oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell)["nnz"]
    assert larger > 0
    As, cfs, _, ells = to_device(ps)
    ncs, nzs = clair.clair_size_R(As, cfs, ells, ctx=ctx)
    assert list(nzs) == [i["nnz"] for i in infos]
    # the FP64 form agrees on the pattern where its 64-vertex search holds the rows
    fp, finfos, st = gpu_build(ps[:3], ctx=ctx, precision=clair.CLAIR_PREC_FP64, check=False)
    for x, y, fi in zip(res, fp, finfos):
        if fi["status"] == 0:
            assert np.array_equal(x["col_idx"], y["col_idx"])


def test_mixed_literal_with_threshold_and_strength_matrix():
    from paper_2307_00229_amd import clair

    from .test_gpu_strength import _dev_csr, _random_graph

    p = P.small_2d(40, stencil=5, eps=0.1, angle=0.5, ell=3)
    ctx = _ctx()
    ctx.set_strength(0.25)
    print("[gpu] literal pattern, theta=0.25, ell=3, mixed form", flush=True)
    res, infos, st = gpu_build([p], ctx=ctx)
    assert st == 0, infos
    o = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, theta=0.25, literal=True)
    assert_matches_oracle(p, res[0], o, infos[0])
    ps = [P.random_sparse(300, 0.01, 41, ell=3), P.small_2d(40, stencil=9, eps=1e-2, angle=0.7, k=3, ell=3)]
    graphs = [_random_graph(q, 7 + k) for k, q in enumerate(ps)]
    ctx = _ctx()
    ctx.set_graph([_dev_csr(*g, n=q.n) for g, q in zip(graphs, ps)])
    print("[gpu] literal pattern on strength matrices, ell=3, mixed form", flush=True)
    res, infos, st = gpu_build(ps, ctx=ctx)
    assert st == 0, infos
    for q, g, gr, inf in zip(ps, res, graphs, infos):
        o = oracle.build_R(q.n, q.row_ptr, q.col_idx, q.val, q.cf, q.B, q.ell, strength=gr, literal=True)
        assert_matches_oracle(q, g, o, inf)


def test_approximate_inverse_build_with_the_literal_pattern():
    from paper_2307_00229_amd import clair

    p = _cases(3)[0]
    A = clair.CSR.from_problem(p, "cuda")
    out, info, _ = clair.clair_build_R_approx(A, torch.from_numpy(p.cf).cuda(), torch.from_numpy(p.B).cuda(),
                                              p.ell, 2, inverse=clair.CLAIR_INVERSE_DIAG, ctx=_ctx())
    rp, ci, va = out
    g = dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(), n_c=info["n_c"],
             nnz=info["nnz"])
    o = oracle.build_R_approx(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, 2, "diag", literal=True)
    assert np.array_equal(g["col_idx"], o["col_idx"])
    assert row_errors(p, g, o)[0].max() <= 1e-10


def test_literal_pattern_with_a_strength_threshold():
    from paper_2307_00229_amd import clair

    p = P.small_2d(40, stencil=5, eps=0.1, angle=0.5, ell=3)
    ctx = _ctx()
    ctx.set_strength(0.25)
    print("[gpu] literal pattern, theta=0.25, ell=3, FP64 form", flush=True)
    res, infos, st = gpu_build([p], ctx=ctx, precision=clair.CLAIR_PREC_FP64)
    assert st == 0, infos
    o = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, theta=0.25, literal=True)
    assert_matches_oracle(p, res[0], o, infos[0])


def test_literal_pattern_on_a_strength_matrix():
    from paper_2307_00229_amd import clair

    from .test_gpu_strength import _dev_csr, _random_graph

    ps = [P.random_sparse(300, 0.01, 41, ell=3), P.small_2d(40, stencil=9, eps=1e-2, angle=0.7, k=3, ell=3)]
    graphs = [_random_graph(p, 7 + k) for k, p in enumerate(ps)]
    ctx = _ctx()
    ctx.set_graph([_dev_csr(*g, n=p.n) for g, p in zip(graphs, ps)])
    print("[gpu] literal pattern on strength matrices, ell=3, FP64 form", flush=True)
    res, infos, st = gpu_build(ps, ctx=ctx, precision=clair.CLAIR_PREC_FP64)
    assert st == 0, infos
    for p, g, gr, inf in zip(ps, res, graphs, infos):
        o = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, strength=gr, literal=True)
        assert_matches_oracle(p, g, o, inf)


def test_flag_values_and_switching_back():
    from paper_2307_00229_amd import clair

    lib = clair.load_library()
    ctx = clair.Context()
    for bad in (2, -1):
        assert lib.clair_ctx_set_literal_pattern(ctx.handle, bad) == clair.CLAIR_ERR_INVALID
    assert lib.clair_ctx_set_literal_pattern(None, 1) == clair.CLAIR_ERR_INVALID
    ps = _cases(3)[:1]
    _, _, st = gpu_build(ps, ctx=ctx, check=False)  # rejected values left the default
    assert st == 0
    a, _, st = gpu_build(ps, ctx=ctx, check=False)
    ctx.set_literal_pattern(True)
    b, _, st2 = gpu_build(ps, ctx=ctx, check=False)
    assert st2 == 0 and b[0]["nnz"] > a[0]["nnz"]
    ctx.set_literal_pattern(False)
    c, _, st3 = gpu_build(ps, ctx=ctx, check=False)
    assert st3 == 0 and np.array_equal(c[0]["col_idx"], a[0]["col_idx"])


@pytest.mark.parametrize("theta", [0.0, 0.3])
def test_literal_pattern_c_points_without_f_neighbours(theta):
    # many C-points, so that some have no (strong) F-neighbour: T's identity
    # part still lets the second step expand them; both forms against the
    # oracle's literal search (pinned against boolean products) at ell = 3
    from paper_2307_00229_amd import clair

    ps = [P.random_sparse(300, 0.01, 60 + k, c_frac=0.55, ell=3) for k in range(2)]
    ctx = _ctx()
    ctx.set_strength(theta)
    for prec in (clair.CLAIR_PREC_FP64, clair.CLAIR_PREC_MIXED):
        print(f"[gpu] literal pattern, dense C-points, theta={theta}, ell=3, precision {prec}", flush=True)
        res, infos, st = gpu_build(ps, ctx=ctx, precision=prec)
        assert st == 0, infos
        for p, g, inf in zip(ps, res, infos):
            o = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, theta=theta, literal=True)
            assert_matches_oracle(p, g, o, inf)
