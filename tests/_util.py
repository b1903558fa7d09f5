"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare it with the oracle.

Comparison rules (derived from the arithmetic, see the parity tests):
* row_ptr and col_idx must be identical (integer work is bit-exact);
* relative row error e_i = max_j |r_gpu - r_orc| / max_j |r_orc| over the
  F-entries of row i, gate 1e-10;
* C-point entries are exactly 1.0;
* constraint residual |sum_i R_ij B_i - B_j| <= 1e-12 * (|B_j| + sum_i |R_ij B_i|)
  on every covered F-column, computed from the GPU result (the rounding error
  of an FP64 sum is relative to the magnitude of its terms);
* n_c, nnz(R) and the number of uncovered F-points equal the oracle's.
"""
from __future__ import annotations

import numpy as np

ROW_TOL = 1e-10
CONSTRAINT_TOL = 1e-12


def to_device(problems, device="cuda"):
    import torch

    from paper_2307_00229_amd import clair

    As = [clair.CSR.from_problem(p, device) for p in problems]
    cfs = [torch.from_numpy(p.cf).to(device) for p in problems]
    Bs = [None if p.B is None else torch.from_numpy(p.B).to(device) for p in problems]
    ells = [p.ell for p in problems]
    return As, cfs, Bs, ells


def gpu_build(problems, **kw):
    from paper_2307_00229_amd import clair

    As, cfs, Bs, ells = to_device(problems)
    outs, infos, st = clair.clair_build_R_batched(As, cfs, Bs, ells, **kw)
    res = []
    for o in outs:
        rp, ci, va = o.trimmed()
        res.append(dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(),
                        n_c=o.n_c, nnz=o.nnz))
    return res, infos, st


def row_errors(p, g, o):
    """Per-row relative error over F-entries (oracle o, GPU g, same pattern)."""
    n_c = o["n_c"]
    C = np.nonzero(p.cf)[0]
    rows = np.repeat(np.arange(n_c), np.diff(o["row_ptr"]))
    fmask = o["col_idx"] != C[rows]
    diff = np.zeros(n_c)
    scale = np.zeros(n_c)
    np.maximum.at(diff, rows[fmask], np.abs(g["val"][fmask] - o["val"][fmask]))
    np.maximum.at(scale, rows[fmask], np.abs(o["val"][fmask]))
    err = np.where(scale > 0, diff / np.where(scale > 0, scale, 1.0), diff)
    return err, fmask, rows


def constraint_residual(p, g):
    C = np.nonzero(p.cf)[0]
    n_c = len(C)
    rows = np.repeat(np.arange(n_c), np.diff(g["row_ptr"]))
    fmask = g["col_idx"] != C[rows]
    cols = g["col_idx"][fmask]
    terms = g["val"][fmask] * p.B[C[rows[fmask]]]
    colsum = np.zeros(p.n)
    colabs = np.zeros(p.n)
    np.add.at(colsum, cols, terms)
    np.add.at(colabs, cols, np.abs(terms))
    covered = np.zeros(p.n, bool)
    covered[cols] = True
    Fc = covered & (p.cf == 0)
    if not Fc.any():
        return 0.0, int(((p.cf == 0) & ~covered).sum())
    # rounding of a sum is relative to the size of its terms
    scale = np.abs(p.B[Fc]) + colabs[Fc]
    return float(np.max(np.abs(colsum[Fc] - p.B[Fc]) / scale)), int(((p.cf == 0) & ~covered).sum())


def assert_matches_oracle(p, g, o, info=None, row_tol=ROW_TOL):
    assert g["n_c"] == o["n_c"], (p.name, g["n_c"], o["n_c"])
    assert g["nnz"] == o["nnz"], (p.name, g["nnz"], o["nnz"])
    assert np.array_equal(g["row_ptr"], o["row_ptr"]), p.name
    assert np.array_equal(g["col_idx"], o["col_idx"]), p.name
    C = np.nonzero(p.cf)[0]
    rows = np.repeat(np.arange(o["n_c"]), np.diff(o["row_ptr"]))
    cmask = o["col_idx"] == C[rows] if o["n_c"] else np.zeros(0, bool)
    assert np.all(g["val"][cmask] == 1.0), p.name
    if o["nnz"]:
        err, _, _ = row_errors(p, g, o)
        worst = float(err.max()) if err.size else 0.0
        assert worst <= row_tol, (p.name, worst, int(err.argmax()))
    if p.B is not None and o["n_c"]:
        res, unc = constraint_residual(p, g)
        assert res <= CONSTRAINT_TOL, (p.name, res)
        assert unc == o["n_uncovered"], (p.name, unc, o["n_uncovered"])
        if info is not None:
            assert info["n_uncovered"] == o["n_uncovered"], (p.name, info["n_uncovered"], o["n_uncovered"])
    if info is not None:
        assert info["status"] == 0, (p.name, info)
        assert info["n_c"] == o["n_c"] and info["nnz"] == o["nnz"]
