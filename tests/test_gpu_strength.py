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
