"""GPU: clair_build_R_noalloc, the entry point for callers that cannot
allocate, against clair_build_R_ex on the same inputs (through the C ABI):
the same sizes and the same bits (both run the same kernels in the same
order), twice in a row with the second matrix smaller, and the oracle's
tolerance.  An input beyond the static scratch is refused before any device
work."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2307_00229_amd import problems as P

from ._util import assert_matches_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(fn_name, p, ctx=None):
    from paper_2307_00229_amd import clair

    lib = clair.load_library()
    A = clair.CSR.from_problem(p, "cuda")
    cf = torch.from_numpy(p.cf).cuda()
    B = torch.from_numpy(p.B).cuda()
    Ac = A.c()
    probe = clair.CsrOut()
    info = clair.Info()
    torch.cuda.synchronize()
    if fn_name == "noalloc":
        st = lib.clair_build_R_noalloc(ctypes.byref(Ac), cf.data_ptr(), B.data_ptr(), p.ell, ctypes.byref(probe), None,
                                       ctypes.byref(info))
    else:
        o = clair.Opts(None, clair.CLAIR_PREC_MIXED, 0, 0, 0)
        st = lib.clair_build_R_ex(ctx.handle, ctypes.byref(Ac), cf.data_ptr(), B.data_ptr(), p.ell,
                                  ctypes.byref(probe), ctypes.byref(o), ctypes.byref(info))
    assert st == clair.CLAIR_ERR_CAPACITY, st  # size query
    out = clair.ROut(int(probe.n_rows), int(probe.nnz), "cuda")
    Rc = out.c()
    free0 = torch.cuda.mem_get_info()[0]
    if fn_name == "noalloc":
        st = lib.clair_build_R_noalloc(ctypes.byref(Ac), cf.data_ptr(), B.data_ptr(), p.ell, ctypes.byref(Rc), None,
                                       ctypes.byref(info))
    else:
        st = lib.clair_build_R_ex(ctx.handle, ctypes.byref(Ac), cf.data_ptr(), B.data_ptr(), p.ell, ctypes.byref(Rc),
                                  ctypes.byref(o), ctypes.byref(info))
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert st == 0, (fn_name, st, clair.load_library().clair_last_error())
    rp, ci, va = out.trimmed()
    g = dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val=va.cpu().numpy(), n_c=out.n_c, nnz=out.nnz)
    return g, info, free0 - free1


def test_noalloc_matches_the_allocating_entry_point_twice():
    from paper_2307_00229_amd import clair

    ctx = clair.Context()
    for p in (P.cfg2(eps_list=(1e-2,))[0],  # 512 x 512: the documented size that fits
              P.small_2d(200, stencil=5, eps=1e-2, angle=0.5, ell=2),  # then smaller ones
              P.small_2d(90, stencil=9, eps=1e-3, angle=2.0, k=3, ell=2)):
        print(f"[gpu] noalloc {p.name}", flush=True)
        rng = np.random.default_rng(p.n)
        p.B = rng.uniform(0.5, 1.5, p.n)
        g0, i0, _ = _run("ex", p, ctx)
        g1, i1, used = _run("noalloc", p)
        assert np.array_equal(g0["row_ptr"], g1["row_ptr"]) and np.array_equal(g0["col_idx"], g1["col_idx"])
        assert np.array_equal(g0["val"].view(np.int64), g1["val"].view(np.int64))
        assert (i0.n_c, i0.nnz, i0.n_uncovered) == (i1.n_c, i1.nnz, i1.n_uncovered)
        assert used == 0  # no device memory taken by the call
        assert_matches_oracle(p, g1, oracle.build_R_problem(p), i1.as_dict())


def test_noalloc_refuses_inputs_beyond_the_scratch():
    from paper_2307_00229_amd import clair

    lib = clair.load_library()
    p = P.small_2d(1200, stencil=5, eps=1e-2, angle=0.5, ell=2)  # 1.44 M fine points: about 290 MB of workspace
    A = clair.CSR.from_problem(p, "cuda")
    cf = torch.from_numpy(p.cf).cuda()
    B = torch.from_numpy(p.B).cuda()
    Ac = A.c()
    out = clair.CsrOut()
    st = lib.clair_build_R_noalloc(ctypes.byref(Ac), cf.data_ptr(), B.data_ptr(), p.ell, ctypes.byref(out), None, None)
    assert st == clair.CLAIR_ERR_UNSUPPORTED
    assert b"static scratch" in lib.clair_last_error()
