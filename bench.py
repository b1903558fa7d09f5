#!/usr/bin/env python3
"""Benchmark: C-l-AIR restriction setup, R rows per second, on one GPU.

One step = the whole setup (neighbourhood search, C/F indexing, block gather,
FP32 factorisation + FP64 refinement, R write, constraint projection) for
every matrix of the workload, inputs resident in HBM.  Default workload: the
batch of 64 5-point upwind advection-diffusion matrices (sides drawn from
64..768, eps log-uniform in [1e-6, 1], random flow angle, ell 1 or 2, seed 0;
3,189,226 rows of R), the largest workload, set up in one batched pass.

Prints one JSON line.  Besides the contract fields it carries
* the plain FP64 per-row form measured on the same inputs and the ratio;
* accuracy gates of the measured result against the FP64 oracle;
* "roofline" for the dominant kernel: the stage with the largest time per
  step (HIP events on the library's stream), with the whole step's fraction
  and a measured device-copy bandwidth beside the 8 TB/s peak;
* "cpu_baseline": the oracle on all host cores, and on one core;
* "plan_numeric_only": repeated setups on a fixed pattern (symbolic phase
  once, numeric phase per step), beside the headline, never as it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "R rows/sec (CℓAIR setup), mixed+batched vs FP64 plain, at ≤1e-10 row error"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "cfg2": "3x 512^2 5-pt upwind adv-diff, eps in {1e-6,1e-2,1}, b=(cos pi/6, sin pi/6), C every 2nd node, ell=2, B=1",
    "cfg1": "32^2 5-pt upwind adv-diff, eps=0.1, C=(even,even), ell=1, B=1",
    "cfg3": "2048^2 9-pt upwind recirculating flow, eps=1e-4, C every 3rd node, ell=2, B=1",
    "cfg4": "64x 5-pt upwind adv-diff, sides U{64..768}, eps 10^U(-6,0), random angle, ell U{1,2}, seed 0, B=1",
    "cfg5": "128^3 7-pt upwind adv-diff, eps=1e-3, b=(1,.5,.25)/|b|, C every 2nd node, ell=2, B=1",
}


def make_problems(name):
    from paper_2307_00229_amd import problems as P

    return {"cfg1": lambda: [P.cfg1()], "cfg2": P.cfg2, "cfg3": lambda: [P.cfg3()], "cfg4": P.cfg4,
            "cfg5": lambda: [P.cfg5()]}[name]()


def algorithmic_bytes(problems, n_c_list, nnz_list):
    """Bytes every implementation must move once: A's CSR, cf, B, R's CSR."""
    whole, kernel = 0, 0
    for p, n_c, nnz in zip(problems, n_c_list, nnz_list):
        a = 4 * (p.n + 1) + 12 * p.nnz
        r = 4 * (n_c + 1) + 12 * nnz
        whole += a + p.n + 8 * p.n + r
        # the numeric kernel reads A once, the C/F marker and B at the C-points,
        # and writes R once
        kernel += a + p.n + 8 * n_c + r
    return whole, kernel


def read_traffic_profile(workload, stage, kernel_src_hash):
    """Counter bytes per launch of a stage's kernel from a committed rocprofv3
    summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{stage}_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_src_sha256") != kernel_src_hash:
        return None
    return d.get("traffic_bytes_per_launch")


def bin_rows(outs, tuning):
    """Rows of R in each size bin of the mixed path: (A) |N| up to the small
    solver's bound, (B) up to 32 points, (C) beyond (the workgroup solver)."""
    import numpy as np

    g = tuning["group"]
    lim = 8 if g <= 4 else g
    a = b = c = 0
    for o in outs:
        s = np.diff(o.trimmed()[0].cpu().numpy()) - 1
        a += int(np.count_nonzero(s <= lim))
        b += int(np.count_nonzero((s > lim) & (s <= 32)))
        c += int(np.count_nonzero(s > 32))
    return a, b, c


def stage_kernel_name(stage, tuning):
    g = tuning["group"]
    small = {1: "k_rows8", 4: "k_quad8"}.get(g, f"k_numeric<{g},...> (bin A)")
    return {"adj": "k_adj", "count": "k_count", "count_mid": "k_count_mid", "count_big": "k_count_big", "scan": "k_scan", "numeric": small,
            "numeric32": "k_numeric<16|32,128,SM> (bin B)", "rows_wg": "k_rows_wg", "project": "k_colproj",
            "upload": "descriptor upload"}.get(stage, stage)


def measure_copy_bandwidth(torch, dev, stream, mib=1024, reps=5):
    """GB/s of a device-to-device copy of `mib` MiB (bytes read + written)."""
    n = mib * 2 ** 20 // 4
    x = torch.ones(n, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    best = float("inf")
    with torch.cuda.stream(stream):
        y.copy_(x)
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            y.copy_(x)
            e1.record(stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / 1e3)
    del x, y
    return 2 * n * 4 / best / 1e9


def kernel_source_hash():
    h = hashlib.sha256()
    for fn in ("k_mixed.hip", "clair_device.h"):
        with open(os.path.join(ROOT, "paper_2307_00229_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(problems, budget_s):
    """The oracle as it stands: the whole workload repeated on all host
    threads for about budget_s, then on one thread over the matrices in turn
    for about budget_s (a bounded sample of the same workload)."""
    import oracle

    nthreads = oracle.max_threads()
    rows = 0
    t0 = time.perf_counter()
    reps = 0
    while True:
        for p in problems:
            o = oracle.build_R_problem(p)
            rows += o["n_c"]
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    rows1, n1 = 0, 0
    t1 = time.perf_counter()
    while True:
        p = problems[n1 % len(problems)]
        rows1 += oracle.build_R_problem(p, nthreads=1)["n_c"]
        n1 += 1
        el1 = time.perf_counter() - t1
        if el1 >= budget_s:
            break
    return dict(value=rows / el, unit="rows/s", cores=nthreads, kind="oracle",
                sample=f"full workload x{reps} ({rows} R rows, {el:.1f} s, OpenMP over rows)",
                single_core={"value": rows1 / el1, "unit": "rows/s", "cores": 1,
                             "sample": f"{n1} matrices of the workload in order ({rows1} R rows, {el1:.1f} s)"},
                cpu_model=cpu_model(), host_threads=os.cpu_count())


def check_against_oracle(problems, outs):
    import numpy as np

    import oracle

    worst_row, worst_c = 0.0, 0.0
    for p, o in zip(problems, outs):
        rp, ci, va = (t.cpu().numpy() for t in o.trimmed())
        ref = oracle.build_R_problem(p)
        if not (np.array_equal(rp, ref["row_ptr"]) and np.array_equal(ci, ref["col_idx"])):
            return dict(pattern_identical=False)
        C = np.nonzero(p.cf)[0]
        rows = np.repeat(np.arange(ref["n_c"]), np.diff(ref["row_ptr"]))
        fm = ci != C[rows]
        diff = np.zeros(ref["n_c"])
        scale = np.zeros(ref["n_c"])
        np.maximum.at(diff, rows[fm], np.abs(va[fm] - ref["val"][fm]))
        np.maximum.at(scale, rows[fm], np.abs(ref["val"][fm]))
        ok = scale > 0
        if ok.any():
            worst_row = max(worst_row, float(np.max(diff[ok] / scale[ok])))
        if p.B is not None:
            terms = va[fm] * p.B[C[rows[fm]]]
            colsum = np.zeros(p.n)
            colabs = np.zeros(p.n)
            np.add.at(colsum, ci[fm], terms)
            np.add.at(colabs, ci[fm], np.abs(terms))
            cov = np.zeros(p.n, bool)
            cov[ci[fm]] = True
            Fc = cov & (p.cf == 0)
            if Fc.any():
                rel = np.abs(colsum[Fc] - p.B[Fc]) / (np.abs(p.B[Fc]) + colabs[Fc])
                worst_c = max(worst_c, float(np.max(rel)))
    return dict(pattern_identical=True, max_row_rel_err=worst_row, max_constraint_resid=worst_c)


def time_next_level(clair, ctx, A, cf, B, ell, R_out, stream, reps=5):
    """A^T, P = W(A) and A_c = R A P on one matrix: C calls into preallocated
    buffers (sizes read once beforehand), wall time of the synchronous call."""
    import ctypes

    import numpy as np
    import torch

    lib = clair.load_library()
    sp_ = clair._stream_ptr(stream)

    def best_of(fn):
        assert fn() == 0
        t = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = fn()
            torch.cuda.synchronize()
            t = min(t, time.perf_counter() - t0)
            assert st == 0
        return t * 1e3

    rp, ci, va = R_out.trimmed()
    R = clair.CSR(rp, ci, va, n=R_out.n_c)
    Ac_, Rc_ = A.c(), R.c()
    T = clair.ROut(A.n, int(A.col_idx.numel()), device=A.row_ptr.device)
    Tc = T.c()
    t_ms = best_of(lambda: lib.clair_transpose(ctx.handle, ctypes.byref(Ac_), A.n, ctypes.byref(Tc), sp_))
    o = clair.Opts(sp_, clair.CLAIR_PREC_MIXED, 0, 0, 0)
    info = clair.Info()
    probe = clair.CsrOut()
    lib.clair_build_P(ctx.handle, ctypes.byref(Ac_), cf.data_ptr(), clair._ptr(B), ell, ctypes.byref(probe),
                      ctypes.byref(o), ctypes.byref(info))
    Pout = clair.ROut(A.n, int(probe.nnz), device=A.row_ptr.device)
    Pc = Pout.c()
    p_ms = best_of(lambda: lib.clair_build_P(ctx.handle, ctypes.byref(Ac_), cf.data_ptr(), clair._ptr(B), ell,
                                             ctypes.byref(Pc), ctypes.byref(o), ctypes.byref(info)))
    n_c = int(Pc.n_cols)
    prp, pci, pva = Pout.trimmed()
    Pm = clair.CSR(prp, pci, pva, n=A.n)
    Pmc = Pm.c()
    probe = clair.CsrOut()
    lib.clair_galerkin(ctx.handle, ctypes.byref(Rc_), ctypes.byref(Ac_), ctypes.byref(Pmc), n_c, ctypes.byref(probe),
                       sp_)
    G = clair.ROut(n_c, int(probe.nnz), device=A.row_ptr.device)
    Gc = G.c()
    g_ms = best_of(lambda: lib.clair_galerkin(ctx.handle, ctypes.byref(Rc_), ctypes.byref(Ac_), ctypes.byref(Pmc),
                                              n_c, ctypes.byref(Gc), sp_))
    Bs_out = torch.empty(A.n, dtype=torch.float64, device=A.row_ptr.device)
    ones = torch.ones(A.n, dtype=torch.float64, device=A.row_ptr.device)
    s_ms = best_of(lambda: lib.clair_smooth_B(ctx.handle, ctypes.byref(Ac_), cf.data_ptr(), ones.data_ptr(),
                                              Bs_out.data_ptr(), 5, 2.0 / 3.0, 1, sp_))
    # four constraint vectors imposed on a copy of R (the projection is idempotent)
    va_k = va.clone()
    Rk = clair.CsrOut(R_out.n_c, A.n, int(ci.numel()), R_out.n_c + 1, 0, int(ci.numel()), rp.data_ptr(),
                      ci.data_ptr(), va_k.data_ptr())
    B4 = torch.from_numpy(np.random.default_rng(4).uniform(0.5, 1.5, (A.n, 4))).to(A.row_ptr.device)
    unc = ctypes.c_int64(0)
    k_ms = best_of(lambda: lib.clair_project_constraints(ctx.handle, ctypes.byref(Rk), A.n, cf.data_ptr(),
                                                         B4.data_ptr(), 4, 1e-12, ctypes.byref(unc), sp_))
    # Algorithm 1 with the diagonal block inverse, three iterations
    info_d = clair.Info()
    probe = clair.CsrOut()
    lib.clair_build_R_diag(ctx.handle, ctypes.byref(Ac_), cf.data_ptr(), clair._ptr(B), ell, 3, ctypes.byref(probe),
                           ctypes.byref(info_d), sp_)
    Dout = clair.ROut(int(probe.n_rows), int(probe.nnz), device=A.row_ptr.device)
    Dc = Dout.c()
    d_ms = best_of(lambda: lib.clair_build_R_diag(ctx.handle, ctypes.byref(Ac_), cf.data_ptr(), clair._ptr(B), ell,
                                                  3, ctypes.byref(Dc), ctypes.byref(info_d), sp_))
    i_ms = best_of(lambda: lib.clair_build_R_approx(ctx.handle, ctypes.byref(Ac_), cf.data_ptr(), clair._ptr(B), ell,
                                                    clair.CLAIR_INVERSE_ILU0, 0, 3, ctypes.byref(Dc),
                                                    ctypes.byref(info_d), sp_))
    m_ms = best_of(lambda: lib.clair_build_R_approx(ctx.handle, ctypes.byref(Ac_), cf.data_ptr(), clair._ptr(B), ell,
                                                    clair.CLAIR_INVERSE_GMRES, 3, 3, ctypes.byref(Dc),
                                                    ctypes.byref(info_d), sp_))
    k2_ms = best_of(lambda: lib.clair_build_R_kkt(ctx.handle, ctypes.byref(Ac_), cf.data_ptr(), clair._ptr(B), ell,
                                                  ctypes.byref(Dc), ctypes.byref(info_d), sp_))
    return {"matrix": "first of the workload", "transpose_ms": t_ms, "build_P_ms": p_ms, "galerkin_ms": g_ms,
            "smooth_B_5_cff_on_AT_ms": s_ms, "project_constraints_k4_ms": k_ms, "build_R_diag_3_iterations_ms": d_ms,
            "build_R_ilu0_3_iterations_ms": i_ms, "build_R_gmres3_3_iterations_ms": m_ms,
            "build_R_kkt_ms": k2_ms, "build_R_kkt_cg_steps": int(info_d.refine_iters_max),
            "nnz_A": int(A.col_idx.numel()), "nnz_P": int(Pc.nnz), "nnz_Ac": int(Gc.nnz),
            "note": "synchronous C calls into preallocated buffers, wall time, best of 5"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="cfg4", choices=sorted(WORKLOADS))
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tuning", default=None,
                    help="fixed tuning GROUP,WG_THREADS,CHUNK[,BINB_LANES] instead of the autotuner's pick")
    ap.add_argument("--aggregates", action="store_true",
                    help="C/F splitting and base pattern from greedy aggregates (clair_build_R_agg); "
                         "direct launches only, no plain form, graph or plan")
    ap.add_argument("--theta", type=float, default=0.0,
                    help="strength threshold of the pattern (0: every stored nonzero)")
    ap.add_argument("--no-plan", action="store_true", help="skip the fixed-pattern (plan) measurement")
    ap.add_argument("--no-next-level", action="store_true",
                    help="skip timing P, the transpose and the Galerkin product on the first matrix")
    ap.add_argument("--mode", choices=["graph", "direct", "best"], default="best")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this size (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); sharding the "
              "setup over several GPUs is not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2307_00229_amd import clair

    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    dev = "cuda:0"
    problems = make_problems(args.workload)
    if args.theta:
        import dataclasses

        problems = [dataclasses.replace(p, theta=args.theta) for p in problems]
    if args.aggregates:
        from paper_2307_00229_amd import problems as P

        problems = [P.greedy_aggregates(p) for p in problems]
    As = [clair.CSR.from_problem(p, dev) for p in problems]
    cfs = [torch.from_numpy(p.cf).to(dev) for p in problems]
    Bs = [torch.from_numpy(p.B).to(dev) for p in problems]
    ells = [p.ell for p in problems]
    stream = torch.cuda.Stream()
    ctx = clair.Context()
    ctx.set_strength(args.theta)
    aggs = [torch.from_numpy(p.agg).to(dev) for p in problems] if args.aggregates else None
    with torch.cuda.stream(stream):
        if aggs is None:
            n_c_list, nnz_list = clair.clair_size_R(As, cfs, ells, ctx=ctx, stream=stream)
        else:
            sized, _, _ = clair.clair_build_R_agg(As, cfs, aggs, Bs, ells, ctx=ctx, stream=stream)
            n_c_list, nnz_list = [o.n_c for o in sized], [o.nnz for o in sized]
        outs = [clair.ROut(nc, nz, dev) for nc, nz in zip(n_c_list, nnz_list)]
        if args.tuning:
            t = [int(x) for x in args.tuning.split(",")]
            ctx.set_tuning(*t[:3])
            if len(t) > 3:
                ctx.set_bin_shape(t[3])
        elif not args.no_autotune and aggs is None:
            clair.clair_autotune(ctx, As, cfs, Bs, ells, outs, reps=3, stream=stream)
        tuning = ctx.get_tuning()
        tuning["binB_lanes"] = ctx.get_bin_shape()
        rows = sum(n_c_list)

        direct_step = clair.BatchedCall(ctx, As, cfs, Bs, ells, outs, async_=True, stream=stream, aggs=aggs)

        graph, graph_error = None, None
        try:
            if aggs is not None:
                raise clair.ClairError(clair.CLAIR_ERR_UNSUPPORTED, "graphs take the classical pattern")
            # capture on a stream of its own: a failed capture must not leave
            # the measurement stream unusable
            cap_stream = torch.cuda.Stream()
            graph = clair.Graph(ctx, As, cfs, Bs, ells, outs, stream=cap_stream)
        except clair.ClairError as e:
            graph_error = str(e)
            print(f"graph capture unavailable: {e}", file=sys.stderr)

        def graph_step():
            graph.launch(stream)

        def timed(step, k, w):
            for _ in range(w):
                step()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record(stream)
            for _ in range(k):
                step()
            e1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            return max(e0.elapsed_time(e1) / 1e3, 1e-12), wall

        modes = {"graph": graph_step, "direct": direct_step}
        results = {}
        names = ["graph", "direct"] if args.mode == "best" else [args.mode]
        if graph is None:
            names = [n for n in names if n != "graph"] or ["direct"]
        for name in names:
            dev_s, wall_s = timed(modes[name], args.steps, args.warmup)
            results[name] = dict(dev_s=dev_s, wall_s=wall_s)
        best = min(results, key=lambda k: results[k]["wall_s"])
        t_mixed = results[best]["wall_s"] / args.steps
        # status of the measured runs
        st, infos = graph.info() if best == "graph" else ctx.info(len(problems), outs)
        assert st == 0, infos

        # dominant kernel: per-stage HIP events on the library's stream
        ctx.stage_times()
        timed_step = clair.BatchedCall(ctx, As, cfs, Bs, ells, outs, async_=True, timing=True, stream=stream,
                                       aggs=aggs)
        for _ in range(args.steps):
            timed_step()
        torch.cuda.synchronize()
        stages = {k: v / args.steps for k, v in ctx.stage_times().items()}

        # plain FP64 per-row form on the same inputs (classical pattern only)
        outs_p, t_plain = None, None
        if aggs is None:
            plain_ctx = clair.Context()
            plain_ctx.set_strength(args.theta)
            outs_p = [clair.ROut(nc, nz, dev) for nc, nz in zip(n_c_list, nnz_list)]

            plain_step = clair.BatchedCall(plain_ctx, As, cfs, Bs, ells, outs_p, precision=clair.CLAIR_PREC_FP64,
                                           async_=False, stream=stream)

            p_dev, p_wall = timed(plain_step, args.plain_steps, 2)
            t_plain = p_wall / args.plain_steps

        # repeated setups on a fixed pattern: symbolic phase once (a plan),
        # numeric phase per step (reported beside the headline, not as it)
        plan_res = None
        if not args.no_plan and aggs is None:
            outs_pl = [clair.ROut(nc, nz, dev) for nc, nz in zip(n_c_list, nnz_list)]
            plan = clair.Plan(ctx, As, cfs, ells, outs_pl, stream=stream)

            def plan_step():
                plan.execute(As, Bs, outs_pl, async_=True, stream=stream)

            pl_dev, pl_wall = timed(plan_step, args.steps, args.warmup)
            st_pl, _ = plan.info()
            assert st_pl == 0
            t_pl = pl_wall / args.steps
            plan_res = {"value": rows / t_pl, "unit": "rows/s", "ms_per_step": t_pl * 1e3,
                        "gates": None, "_outs": outs_pl}

        # the rest of a two-level setup on the first matrix (synchronous calls):
        # A^T, P = W(A), and A_c = R A P with the R measured above
        next_level = None
        if not args.no_next_level and aggs is None:
            next_level = time_next_level(clair, ctx, As[0], cfs[0], Bs[0], ells[0], outs[0], stream)

        if args.copy_probe_mib:
            x = torch.empty(args.copy_probe_mib * 2 ** 20 // 4, dtype=torch.float32, device=dev).fill_(1.0)
            y = torch.empty_like(x)
            torch.cuda.synchronize()
            y.copy_(x)
            torch.cuda.synchronize()

        # achievable HBM bandwidth on this device: a 1 GiB device-to-device
        # copy (read + write), best of 5, events on the same stream
        copy_gbs = measure_copy_bandwidth(torch, dev, stream)

    gates = check_against_oracle(problems, outs)
    if plan_res is not None:
        plan_res["gates"] = check_against_oracle(problems, plan_res.pop("_outs"))
    gates_plain = check_against_oracle(problems, outs_p) if outs_p is not None else None

    whole_bytes, _ = algorithmic_bytes(problems, n_c_list, nnz_list)
    # units per launch: the rows each stage processes (the solvers take the
    # rows of their size bin; every other stage passes over all rows)
    bins = bin_rows(outs, tuning)
    per_row = whole_bytes / rows
    stage_units = {"numeric": bins[0], "numeric32": bins[1], "rows_wg": bins[2], "count_big": bins[2]}
    dom = max(stages, key=stages.get) if stages else None
    t_kern = stages[dom] / 1e3 if dom else float("nan")
    units = stage_units.get(dom, rows)
    kern_bytes = per_row * units
    achieved = kern_bytes / t_kern / 1e9 if t_kern > 0 else None
    src_hash = kernel_source_hash()
    # the committed counters were taken at theta = 0
    traffic = (read_traffic_profile(args.workload, dom, src_hash)
               if (dom and args.theta == 0 and not args.aggregates) else None)
    roofline = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=(achieved / HBM_PEAK_GBS) if achieved else None, traffic=traffic,
                    kernel=stage_kernel_name(dom, tuning), stage=dom, kernel_ms=t_kern * 1e3,
                    rows_per_launch=units, algorithmic_bytes_per_row=per_row,
                    algorithmic_bytes_per_launch=kern_bytes,
                    step_algorithmic_bytes=whole_bytes, step_GBps=whole_bytes / t_mixed / 1e9,
                    step_frac=whole_bytes / t_mixed / 1e9 / HBM_PEAK_GBS,
                    measured_copy_GBps=copy_gbs,
                    step_frac_of_measured_copy=(whole_bytes / t_mixed / 1e9 / copy_gbs) if copy_gbs else None,
                    rows_by_bin=dict(A=bins[0], B=bins[1], C=bins[2]), stage_ms=stages)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(problems, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": rows / t_mixed,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "matrices": len(problems),
                   "R_rows": rows, "nnz_R": int(sum(nnz_list)), "launch": best, "tuning": tuning,
                   "theta": args.theta, "aggregates": bool(args.aggregates),
                   "parallelism": "single GPU"},
        "plain_fp64": ({"value": rows / t_plain, "unit": "rows/s", "ms_per_step": t_plain * 1e3,
                        "gates": gates_plain} if t_plain else None),
        "speedup_vs_plain_fp64": (t_plain / t_mixed) if t_plain else None,
        "plan_numeric_only": plan_res,
        "next_level": next_level,
        "modes_ms_per_step": {k: v["wall_s"] / args.steps * 1e3 for k, v in results.items()},
        "graph_error": graph_error,
        "gates": gates,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
