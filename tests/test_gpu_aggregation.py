"""GPU parity with the aggregation-based base pattern.

clair_build_R_agg (T = the aggregation operator, Section 3.1.3) against the
oracle with the same aggregates (pinned in tests/test_oracle_aggregation.py):
identical pattern, row error <= 1e-10, constraint residual <= 1e-12.  Greedy
aggregates of several matrices, ell = 1..3, with and without a strength
threshold, a batch mixing aggregated and classical matrices, rows above 32
points, and a 512^2 matrix at full size.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2307_00229_amd import problems as P

from ._util import assert_matches_oracle, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_00229_amd import clair

    clair.load_library()


def _run(ps, theta=0.0):
    from paper_2307_00229_amd import clair

    ctx = clair.Context()
    ctx.set_strength(theta)
    As, cfs, Bs, ells = to_device(ps)
    aggs = [None if p.agg is None else torch.from_numpy(p.agg).cuda() for p in ps]
    print(f"[gpu] aggregates {[p.name for p in ps]} theta={theta}", flush=True)
    outs, infos, st = clair.clair_build_R_agg(As, cfs, aggs, Bs, ells, ctx=ctx)
    assert st == 0, infos
    for p, o, inf in zip(ps, outs, infos):
        rp, ci, va = o.trimmed()
        g = dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(), n_c=o.n_c, nnz=o.nnz)
        q = dataclasses.replace(p, theta=theta)
        assert_matches_oracle(q, g, oracle.build_R_problem(q), inf)
    return infos


def _cases(ell):
    return [P.greedy_aggregates(P.small_2d(60, stencil=5, eps=0.05, angle=0.5, ell=ell)),
            P.greedy_aggregates(P.small_2d(48, stencil=9, eps=1e-3, angle=2.0, ell=ell)),
            P.greedy_aggregates(P.small_3d(14, eps=0.05, b=(1.0, 0.3, -0.2), ell=ell)),
            P.greedy_aggregates(P.random_sparse(800, 0.004, 17, ell=ell))]


@pytest.mark.parametrize("theta", [0.0, 0.25])
@pytest.mark.parametrize("ell", [1, 2, 3])
def test_aggregation_parity(ell, theta):
    infos = _run(_cases(ell), theta)
    if ell == 3 and theta == 0.0:
        assert max(i["max_block"] for i in infos) > 32  # the workgroup search took part


def test_batch_mixing_aggregated_and_classical():
    ps = _cases(2)
    ps[1] = dataclasses.replace(ps[1], agg=None, cf=P.small_2d(48, stencil=9, eps=1e-3, angle=2.0, k=3, ell=2).cf)
    _run(ps)


def test_aggregation_512_full_size():
    p = P.greedy_aggregates(P.cfg2()[1])
    infos = _run([p])
    assert infos[0]["n_c"] == int(p.cf.sum())


def test_fp64_form_rejects_aggregates():
    from paper_2307_00229_amd import clair

    p = _cases(2)[0]
    As, cfs, Bs, ells = to_device([p])
    lib = clair.load_library()
    import ctypes

    nm, Ac, cfp, Bp, ellv, Rc = clair._batch_args(As, cfs, Bs, ells, [clair.ROut(0, 0)])
    agg = torch.from_numpy(p.agg).cuda()
    aggp = (ctypes.c_void_p * 1)(agg.data_ptr())
    o = clair.Opts(None, clair.CLAIR_PREC_FP64, 0, 0, 0)
    st = lib.clair_build_R_agg(clair.Context().handle, 1, Ac, cfp, aggp, Bp, ellv, Rc, ctypes.byref(o), None)
    assert st == clair.CLAIR_ERR_UNSUPPORTED


def test_aggregation_with_a_strength_matrix():
    # aggregates give T, a strength matrix of the caller's gives the expansion
    from paper_2307_00229_amd import clair

    from .test_gpu_strength import _dev_csr, _random_graph

    ps = _cases(2)[:2]
    graphs = [_random_graph(p, 51 + k) for k, p in enumerate(ps)]
    ctx = clair.Context()
    ctx.set_graph([_dev_csr(*g, n=p.n) for g, p in zip(graphs, ps)])
    As, cfs, Bs, ells = to_device(ps)
    aggs = [torch.from_numpy(p.agg).cuda() for p in ps]
    outs, infos, st = clair.clair_build_R_agg(As, cfs, aggs, Bs, ells, ctx=ctx)
    assert st == 0, infos
    for p, o, inf, g in zip(ps, outs, infos, graphs):
        rp, ci, va = o.trimmed()
        got = dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(), n_c=o.n_c, nnz=o.nnz)
        ref = oracle.build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, p.B, p.ell, agg=p.agg, strength=g)
        assert_matches_oracle(p, got, ref, inf)
