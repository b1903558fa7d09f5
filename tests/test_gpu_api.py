"""GPU tests of the entry points around the setup: asynchronous calls,
hipGraph replay, size queries and capacity errors, device-side validation,
singular blocks, per-stage timing, the autotuner, and the symbolic/numeric
split (plans)."""
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


def _fetch(o):
    rp, ci, va = o.trimmed()
    return dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(), n_c=o.n_c, nnz=o.nnz)


def _cases():
    return [P.small_2d(200, stencil=5, eps=1e-3, angle=0.5, ell=2),
            P.small_2d(150, stencil=9, eps=0.1, angle=3.0, k=3, ell=2),
            P.small_3d(24, eps=1e-2, b=(1.0, 0.5, 0.25), ell=2)]


def test_async_then_ctx_info():
    from paper_2307_00229_amd import clair

    ps = _cases()
    As, cfs, Bs, ells = to_device(ps)
    ctx = clair.Context()
    ncs, nzs = clair.clair_size_R(As, cfs, ells, ctx=ctx)
    outs = [clair.ROut(a, b) for a, b in zip(ncs, nzs)]
    s = torch.cuda.Stream()
    print("[gpu] async enqueue", flush=True)
    for _ in range(3):
        clair.clair_build_R_batched(As, cfs, Bs, ells, ctx=ctx, outs=outs, async_=True, stream=s)
    st, infos = ctx.info(len(ps), outs)
    assert st == 0, infos
    for p, o, inf in zip(ps, outs, infos):
        assert_matches_oracle(p, _fetch(o), oracle.build_R_problem(p), inf)


def test_async_after_smaller_blocks_uses_workgroup_fallback():
    # the 32-lane solver's block bound follows the last batch whose sizes were
    # read back (here |N| <= 16); an asynchronous call on larger blocks (3D,
    # |N| = 18) hands them to the workgroup solver and stays exact
    from paper_2307_00229_amd import clair

    small = [P.small_2d(120, stencil=9, eps=0.05, angle=1.0, k=2, ell=2)]
    big = [P.small_3d(20, eps=1e-2, b=(1.0, 0.5, 0.25), ell=2)]
    ctx = clair.Context()
    A2, c2, B2, l2 = to_device(big)
    ncs, nzs = clair.clair_size_R(A2, c2, l2, ctx=ctx)
    outs = [clair.ROut(a, b) for a, b in zip(ncs, nzs)]
    A1, c1, B1, l1 = to_device(small)
    _, infos, st = clair.clair_build_R_batched(A1, c1, B1, l1, ctx=ctx)
    assert st == 0 and 8 < infos[0]["max_block"] <= 16, infos
    clair.clair_build_R_batched(A2, c2, B2, l2, ctx=ctx, outs=outs, async_=True)
    st, infos = ctx.info(1, outs)
    assert st == 0, infos
    assert infos[0]["max_block"] == 18
    assert_matches_oracle(big[0], _fetch(outs[0]), oracle.build_R_problem(big[0]), infos[0])


def test_graph_replay_matches_eager():
    from paper_2307_00229_amd import clair

    ps = _cases()
    As, cfs, Bs, ells = to_device(ps)
    ctx = clair.Context()
    eager, _, _ = clair.clair_build_R_batched(As, cfs, Bs, ells, ctx=ctx)
    ref = [_fetch(o) for o in eager]
    outs = [clair.ROut(o.n_c, o.nnz) for o in eager]
    s = torch.cuda.Stream()
    print("[gpu] graph capture", flush=True)
    g = clair.Graph(ctx, As, cfs, Bs, ells, outs, stream=s)
    for rep in range(4):
        for o in outs:
            o.val.fill_(-7.0)
            o.col_idx.fill_(-1)
        torch.cuda.synchronize()
        g.launch(s)
        s.synchronize()
        st, infos = g.info()
        assert st == 0, infos
        # eager work between replays
        clair.clair_build_R_batched(As, cfs, Bs, ells, ctx=ctx)
        for r, o, inf in zip(ref, outs, infos):
            got = _fetch(o)
            assert np.array_equal(got["row_ptr"], r["row_ptr"]) and np.array_equal(got["col_idx"], r["col_idx"])
            np.testing.assert_allclose(got["val"], r["val"], rtol=1e-13, atol=1e-15)
            assert inf["nnz"] == r["nnz"]
    # new values in A (same pattern) flow into the next replay
    for a in As:
        a.val.mul_(3.0)
    g.launch(s)
    s.synchronize()
    for p, o in zip(ps, outs):
        q = P.Problem(p.name, p.n, p.row_ptr, p.col_idx, p.val * 3.0, p.cf, p.B, p.ell)
        assert_matches_oracle(q, _fetch(o), oracle.build_R_problem(q))
    g.close()


def test_size_query_and_capacity_error():
    from paper_2307_00229_amd import clair

    p = P.cfg1()
    As, cfs, Bs, ells = to_device([p])
    ctx = clair.Context()
    small = [clair.ROut(256, 100)]
    outs, infos, st = clair.clair_build_R_batched(As, cfs, Bs, ells, ctx=ctx, outs=small, check=False)
    assert st == clair.CLAIR_ERR_CAPACITY
    assert infos[0]["nnz"] == 1248 and infos[0]["n_c"] == 256
    short_rows = [clair.ROut(10, 5000)]
    outs, infos, st = clair.clair_build_R_batched(As, cfs, Bs, ells, ctx=ctx, outs=short_rows, check=False)
    assert st == clair.CLAIR_ERR_CAPACITY
    # one matrix too small in a batch does not stop the others
    ps = [p, P.small_2d(40, ell=2)]
    As2, cfs2, Bs2, ells2 = to_device(ps)
    ncs, nzs = clair.clair_size_R(As2, cfs2, ells2, ctx=ctx)
    outs = [clair.ROut(ncs[0], 10), clair.ROut(ncs[1], nzs[1])]
    outs, infos, st = clair.clair_build_R_batched(As2, cfs2, Bs2, ells2, ctx=ctx, outs=outs, check=False)
    assert st == clair.CLAIR_ERR_CAPACITY
    assert infos[0]["status"] == clair.CLAIR_ERR_CAPACITY and infos[1]["status"] == 0
    assert_matches_oracle(ps[1], _fetch(outs[1]), oracle.build_R_problem(ps[1]))


def test_validation_rejects_unsorted_and_out_of_range():
    from paper_2307_00229_amd import clair

    p = P.small_2d(16, ell=2)
    ci = p.col_idx.copy()
    ci[1], ci[2] = ci[2], ci[1]
    q = P.Problem("unsorted", p.n, p.row_ptr, ci, p.val, p.cf, p.B, 2)
    r = P.Problem("range", p.n, p.row_ptr, np.where(np.arange(len(ci)) == 7, p.n + 5, p.col_idx).astype(np.int32),
                  p.val, p.cf, p.B, 2)
    As, cfs, Bs, ells = to_device([q, r, p])
    ctx = clair.Context()
    outs = [clair.ROut(p.n, 20 * p.n) for _ in range(3)]
    outs, infos, st = clair.clair_build_R_batched(As, cfs, Bs, ells, ctx=ctx, outs=outs, validate=True, check=False)
    assert infos[0]["status"] == clair.CLAIR_ERR_INVALID and infos[0]["first_bad_row"] == 0
    assert infos[1]["status"] == clair.CLAIR_ERR_INVALID
    assert infos[2]["status"] == 0
    assert_matches_oracle(p, _fetch(outs[2]), oracle.build_R_problem(p))


def test_bad_arguments_rejected_on_host():
    from paper_2307_00229_amd import clair

    p = P.small_2d(8, ell=1)
    As, cfs, Bs, ells = to_device([p])
    with pytest.raises(clair.ClairError) as e:
        clair.clair_build_R_batched(As, cfs, Bs, [0], outs=[clair.ROut(16, 100)])
    assert e.value.status == clair.CLAIR_ERR_INVALID


@pytest.mark.parametrize("precision", [0, 1])
def test_singular_block_reported(precision):
    from paper_2307_00229_amd import clair

    n = 3
    p = P.Problem("sing", n, np.array([0, 3, 6, 9], np.int32), np.array([0, 1, 2] * 3, np.int32),
                  np.array([4.0, -1.0, -1.0, -1.0, 1.0, 1.0, -1.0, 1.0, 1.0]), np.array([1, 0, 0], np.int8), None, 1)
    As, cfs, Bs, ells = to_device([p])
    outs, infos, st = clair.clair_build_R_batched(As, cfs, Bs, ells, outs=[clair.ROut(1, 3)], precision=precision,
                                                  check=False)
    assert st == clair.CLAIR_ERR_SINGULAR
    assert infos[0]["first_bad_row"] == 0


def test_stage_timing_and_autotune():
    from paper_2307_00229_amd import clair

    ps = _cases()
    As, cfs, Bs, ells = to_device(ps)
    ctx = clair.Context()
    ncs, nzs = clair.clair_size_R(As, cfs, ells, ctx=ctx)
    outs = [clair.ROut(a, b) for a, b in zip(ncs, nzs)]
    tuning = clair.clair_autotune(ctx, As, cfs, Bs, ells, outs, reps=1)
    assert tuning["group"] in (1, 4, 8, 16, 32)
    for p, o in zip(ps, outs):
        assert_matches_oracle(p, _fetch(o), oracle.build_R_problem(p))
    ctx.stage_times()
    for _ in range(2):
        clair.clair_build_R_batched(As, cfs, Bs, ells, ctx=ctx, outs=outs, timing=True)
    t = ctx.stage_times()
    assert {"count", "scan", "numeric", "project"} <= set(t)
    assert all(v >= 0 for v in t.values())


@pytest.mark.parametrize("which", ["cfg1", "mixed_bins", "cfg2_eps1e-2"])
def test_repeat_runs_bitwise_identical(which):
    # the projection orders every column's entries by row before summing
    # (Algorithm 1's projection step, one F-column at a time): repeat runs give
    # the same bits, also with random B, rows in several size bins and
    # columns of more than eight rows (the distance-3 random pattern)
    from paper_2307_00229_amd import clair

    if which == "cfg1":
        ps = [P.cfg1()]
    elif which == "mixed_bins":
        ps = _cases() + [P.random_sparse(400, 0.012, 77, ell=3)]
        rng = np.random.default_rng(5)
        for q in ps:
            q.B = rng.uniform(0.5, 1.5, q.n)
    else:
        ps = [P.cfg2(eps_list=(1e-2,))[0]]
    As, cfs, Bs, ells = to_device(ps)
    runs = []
    for _ in range(3):
        outs, infos, st = clair.clair_build_R_batched(As, cfs, Bs, ells, ctx=clair.Context())
        assert st == 0, infos
        runs.append([_fetch(o) for o in outs])
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            assert np.array_equal(a["row_ptr"], b["row_ptr"]) and np.array_equal(a["col_idx"], b["col_idx"])
            assert np.array_equal(a["val"].view(np.int64), b["val"].view(np.int64))
    for q, g in zip(ps, runs[0]):
        assert_matches_oracle(q, g, oracle.build_R_problem(q))


# ---------------------------------------------------------------------------
# symbolic/numeric split (clair_plan_*)
# ---------------------------------------------------------------------------

def _same_pattern_new_values():
    # same grids, stencils and flow directions (so the same upwind pattern),
    # other diffusion constants; random B
    old = _cases()
    new = [P.small_2d(200, stencil=5, eps=0.3, angle=0.5, ell=2),
           P.small_2d(150, stencil=9, eps=1e-3, angle=3.0, k=3, ell=2),
           P.small_3d(24, eps=1.0, b=(1.0, 0.5, 0.25), ell=2)]
    rng = np.random.default_rng(11)
    for a, b in zip(old, new):
        assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col_idx, b.col_idx)
        b.B = rng.uniform(0.5, 1.5, b.n)
    return old, new


def test_plan_execute_matches_full_setup_on_new_values():
    from paper_2307_00229_amd import clair

    old, new = _same_pattern_new_values()
    A0, c0, B0, l0 = to_device(old)
    ctx = clair.Context()
    ncs, nzs = clair.clair_size_R(A0, c0, l0, ctx=ctx)
    outs = [clair.ROut(a, b) for a, b in zip(ncs, nzs)]
    print("[gpu] plan create", flush=True)
    plan = clair.Plan(ctx, A0, c0, l0, outs)
    assert [o.n_c for o in outs] == ncs and [o.nnz for o in outs] == nzs
    infos, st = plan.execute(A0, B0)
    for p, o, inf in zip(old, outs, infos):
        assert_matches_oracle(p, _fetch(o), oracle.build_R_problem(p), inf)
    # new values and B on the same pattern, twice, into fresh R buffers
    A1, _, B1, _ = to_device(new)
    outs1 = [clair.ROut(a, b) for a, b in zip(ncs, nzs)]
    for _ in range(2):
        infos, st = plan.execute(A1, B1, outs1)
        for p, o, inf in zip(new, outs1, infos):
            assert_matches_oracle(p, _fetch(o), oracle.build_R_problem(p), inf)
    # unconstrained rows
    infos, st = plan.execute(A1, None, outs1)
    for p, o in zip(new, outs1):
        q = dataclasses.replace(p, B=None)
        assert_matches_oracle(q, _fetch(o), oracle.build_R_problem(q))
    plan.close()


def test_plan_async_execute_and_info():
    from paper_2307_00229_amd import clair

    old, new = _same_pattern_new_values()
    A0, c0, B0, l0 = to_device(old)
    A1, _, B1, _ = to_device(new)
    ctx = clair.Context()
    ncs, nzs = clair.clair_size_R(A0, c0, l0, ctx=ctx)
    outs = [clair.ROut(a, b) for a, b in zip(ncs, nzs)]
    plan = clair.Plan(ctx, A0, c0, l0, outs)
    s = torch.cuda.Stream()
    for k in range(4):
        plan.execute(A1 if k % 2 else A0, B1 if k % 2 else B0, async_=True, stream=s)
    st, infos = plan.info()
    assert st == 0, infos
    for p, o, inf in zip(new, outs, infos):
        assert_matches_oracle(p, _fetch(o), oracle.build_R_problem(p), inf)


def test_plan_with_workgroup_rows_and_bad_arguments():
    from paper_2307_00229_amd import clair

    # neighbourhoods up to 40 points: rows queued for the workgroup solver by
    # the symbolic phase must be solved again on every execute
    p = P.cfg3(N=90, ell=3)
    As, cfs, Bs, ells = to_device([p])
    ctx = clair.Context()
    ncs, nzs = clair.clair_size_R(As, cfs, ells, ctx=ctx)
    outs = [clair.ROut(ncs[0], nzs[0])]
    plan = clair.Plan(ctx, As, cfs, ells, outs)
    ref = oracle.build_R_problem(p)
    for _ in range(3):
        infos, st = plan.execute(As, Bs)
        assert infos[0]["max_block"] > 32
        assert_matches_oracle(p, _fetch(outs[0]), ref, infos[0])
    # another size than planned, or too small R: rejected before any work
    q = P.cfg3(N=60, ell=3)
    Aq, _, Bq, _ = to_device([q])
    infos, st = plan.execute(Aq, Bq, check=False)
    assert st == clair.CLAIR_ERR_INVALID
    infos, st = plan.execute(As, Bs, [clair.ROut(ncs[0], nzs[0] - 1)], check=False)
    assert st == clair.CLAIR_ERR_CAPACITY


def test_autotune_cache_by_histogram():
    # the pick is cached by (device, block-size histogram signature): a second
    # autotune on the same inputs (another context) makes no timing runs and
    # returns the same tuning; another histogram is timed
    from paper_2307_00229_amd import clair

    ps = [P.small_2d(143, stencil=9, eps=2e-3, angle=1.3, k=3, ell=2), P.small_3d(17, eps=0.02, ell=2)]
    As, cfs, Bs, ells = to_device(ps)
    ncs, nzs = clair.clair_size_R(As, cfs, ells)
    outs = [clair.ROut(a, b) for a, b in zip(ncs, nzs)]
    t1 = clair.clair_autotune(clair.Context(), As, cfs, Bs, ells, outs, reps=1)
    assert t1["timing_runs"] > 0
    ctx2 = clair.Context()
    t2 = clair.clair_autotune(ctx2, As, cfs, Bs, ells, outs, reps=1)
    assert t2["timing_runs"] == 0
    assert {k: t1[k] for k in ("group", "wg_threads", "chunk", "binB_lanes")} == \
        {k: t2[k] for k in ("group", "wg_threads", "chunk", "binB_lanes")}
    for p, o in zip(ps, outs):
        assert_matches_oracle(p, _fetch(o), oracle.build_R_problem(p))
    q = [P.small_2d(61, stencil=5, eps=1e-5, angle=4.0, ell=1)]
    Aq, cq, Bq, eq = to_device(q)
    nq, zq = clair.clair_size_R(Aq, cq, eq)
    oq = [clair.ROut(a, b) for a, b in zip(nq, zq)]
    t3 = clair.clair_autotune(ctx2, Aq, cq, Bq, eq, oq, reps=1)
    assert t3["timing_runs"] > 0
