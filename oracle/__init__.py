"""Oracle for the C-l-AIR restriction setup -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 CPU implementations that the GPU library is checked
against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import this package; the product path never does.  It shares no code with
the GPU library: the C oracle (``clair_oracle.c``) is built with gcc, and the
NumPy modules (``dense``, ``literal``) use only NumPy/SciPy primitives.

Modules
-------
``build_R``      -- ctypes wrapper around the C oracle (closed form of
                    Algorithm 1 with exact local inverses, k = 1).
``dense``        -- brute force on tiny inputs: neighbourhoods by dense
                    boolean reachability, per-row dense solves, and the ideal
                    restriction R_ideal = [-A_cf A_ff^{-1}, I].
``literal``      -- Algorithm 1 step by step (tentative operator, least-squares
                    constraint fit, residual update, explicit projection), for
                    any number k of iterations.
``smoothing``    -- CFF-weighted-Jacobi smoothing of the constraint vector.
``kkt``          -- the exact minimiser in the normal-equations metric (the
                    KKT system of Section 3.1.1), for comparison.
``build_R_approx`` -- Algorithm 1 with approximate block inverses (diagonal,
                    ILU(0) or GMRES) and any number of iterations (C oracle, on the
                    exact build's pattern); ``build_R_diag`` the diagonal one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "clair_oracle.c")
_LIB = os.path.join(_HERE, "libclair_oracle.so")

ORC_OK, ORC_ERR_INVALID, ORC_ERR_CAPACITY, ORC_ERR_SINGULAR, ORC_ERR_NOMEM = 0, 1, 2, 3, 4

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        f64 = ctypes.c_double
        lib.orc_pattern_size.argtypes = [i32, p, p, p, p, p, i32, f64, i32, p, p, p]
        lib.orc_pattern_size.restype = ctypes.c_int
        lib.orc_build_R.argtypes = [i32, p, p, p, p, p, p, i32, f64, i32, p, p, p, i64, p, p]
        lib.orc_build_R.restype = ctypes.c_int
        lib.orc_build_R_g.argtypes = [i32, p, p, p, p, p, p, p, p, p, i32, f64, i32, i32, p, p, p, i64, p, p]
        lib.orc_pattern_size_g.argtypes = [i32, p, p, p, p, p, i32, f64, i32, i32, p, p, p]
        lib.orc_pattern_size_g.restype = ctypes.c_int
        lib.orc_build_R_g.restype = ctypes.c_int
        lib.orc_project_k.argtypes = [i32, i32, p, p, p, p, p, i32, f64, p]
        lib.orc_project_k.restype = ctypes.c_int
        lib.orc_iterate_approx.argtypes = [i32, p, p, p, p, p, i32, p, p, p, i32, i32, i32, p]
        lib.orc_iterate_approx.restype = ctypes.c_int
        lib.orc_max_threads.argtypes = []
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


def max_threads() -> int:
    return int(_load().orc_max_threads())


def pattern_size(n, row_ptr, col_idx, val, cf, ell, nthreads=0, theta=0.0, agg=None, literal=False):
    """(n_c, nnz_R, sizes[n_c]) with sizes[r] = |N(i_r)|.  theta: strength
    threshold; agg: root C-point of every point's aggregate (or -1), for the
    aggregation-based base pattern."""
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col_idx, np.int32)
    va = np.ascontiguousarray(val, np.float64)
    cf = np.ascontiguousarray(cf, np.int8)
    ag = None if agg is None else np.ascontiguousarray(agg, np.int32)
    n_c = ctypes.c_int32(0)
    nnz = ctypes.c_int64(0)
    sizes = np.zeros(int((cf != 0).sum()) or 1, np.int32)
    rc = lib.orc_pattern_size_g(n, _ptr(rp), _ptr(ci), _ptr(va), _ptr(cf), _ptr(ag), ell, float(theta),
                                int(bool(literal)), nthreads, ctypes.byref(n_c), ctypes.byref(nnz), _ptr(sizes))
    if rc:
        raise OracleError(rc, f"oracle pattern_size failed ({rc})")
    return n_c.value, nnz.value, sizes[: n_c.value]


def build_R(n, row_ptr, col_idx, val, cf, B, ell, nthreads=0, allow_singular=False, theta=0.0, agg=None,
            strength=None, literal=False):
    """FP64 oracle R (CSR arrays) plus statistics.  theta: strength threshold
    of the pattern (0 keeps every stored nonzero).  strength: an optional n x n
    CSR (row_ptr, col_idx, val) whose stored entries u -> v are the edges of
    the neighbourhood search instead of A's (theta then filters its entries);
    the local systems always use A.  literal: the pattern of S^{ell-1} T
    taken literally (C-points may be interior vertices of a walk; the same
    as the default for ell <= 2).

    Returns dict(row_ptr, col_idx, val, n_c, nnz, n_uncovered, bad_row).
    """
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col_idx, np.int32)
    va = np.ascontiguousarray(val, np.float64)
    cfa = np.ascontiguousarray(cf, np.int8)
    Ba = None if B is None else np.ascontiguousarray(B, np.float64)
    ag = None if agg is None else np.ascontiguousarray(agg, np.int32)
    if strength is None:
        grp, gci, gva = rp, ci, va
    else:
        grp = np.ascontiguousarray(strength[0], np.int32)
        gci = np.ascontiguousarray(strength[1], np.int32)
        gva = np.ascontiguousarray(strength[2], np.float64)
    n_c, nnz, _ = pattern_size(n, grp, gci, gva, cfa, ell, nthreads, theta=theta, agg=ag, literal=literal)
    Rrp = np.zeros(n_c + 1, np.int32)
    Rci = np.zeros(max(nnz, 1), np.int32)
    Rva = np.zeros(max(nnz, 1), np.float64)
    unc = ctypes.c_int64(0)
    bad = ctypes.c_int32(-1)
    rc = lib.orc_build_R_g(n, _ptr(rp), _ptr(ci), _ptr(va), _ptr(grp), _ptr(gci), _ptr(gva), _ptr(cfa), _ptr(ag),
                           _ptr(Ba), ell, float(theta), int(bool(literal)), nthreads, _ptr(Rrp), _ptr(Rci),
                           _ptr(Rva), nnz,
                           ctypes.byref(unc), ctypes.byref(bad))
    if rc and not (rc == ORC_ERR_SINGULAR and allow_singular):
        raise OracleError(rc, f"oracle build_R failed ({rc}), bad_row={bad.value}")
    return dict(row_ptr=Rrp, col_idx=Rci[:nnz], val=Rva[:nnz], n_c=n_c, nnz=nnz,
                n_uncovered=unc.value, bad_row=bad.value, status=rc)


def build_R_problem(p, nthreads=0, B="problem", **kw):
    """Convenience: oracle R for a problems.Problem."""
    Bv = p.B if (isinstance(B, str) and B == "problem") else B
    kw.setdefault("theta", getattr(p, "theta", 0.0))
    kw.setdefault("agg", getattr(p, "agg", None))
    return build_R(p.n, p.row_ptr, p.col_idx, p.val, p.cf, Bv, p.ell, nthreads=nthreads, **kw)


def build_R_diag(n, row_ptr, col_idx, val, cf, B, ell, iterations, theta=0.0, agg=None):
    """Algorithm 1 with the diagonal block inverse (see build_R_approx)."""
    return build_R_approx(n, row_ptr, col_idx, val, cf, B, ell, iterations, "diag", theta=theta, agg=agg)


def build_R_approx(n, row_ptr, col_idx, val, cf, B, ell, iterations, inverse, theta=0.0, agg=None, krylov=0,
                   strength=None, literal=False):
    """Algorithm 1 with approximate block inverses ("diag": the diagonal of
    each block; "ilu0": its incomplete LU factorisation without fill;
    "gmres": `krylov` steps of GMRES on each local system from zero) and
    `iterations` steps, on the pattern of the exact build (the pattern does
    not depend on the inverse).  Returns the same dict as build_R."""
    lib = _load()
    o = build_R(n, row_ptr, col_idx, val, cf, None, ell, allow_singular=True, theta=theta, agg=agg,
                strength=strength, literal=literal)
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col_idx, np.int32)
    va = np.ascontiguousarray(val, np.float64)
    cfa = np.ascontiguousarray(cf, np.int8)
    Ba = None if B is None else np.ascontiguousarray(B, np.float64)
    Rva = np.zeros(max(o["nnz"], 1), np.float64)
    bad = ctypes.c_int32(-1)
    kind = {"diag": 1, "ilu0": 2, "gmres": 3}[inverse]
    rc = lib.orc_iterate_approx(n, _ptr(rp), _ptr(ci), _ptr(va), _ptr(cfa), _ptr(Ba), o["n_c"], _ptr(o["row_ptr"]),
                                _ptr(np.ascontiguousarray(o["col_idx"], np.int32)), _ptr(Rva), kind, int(krylov),
                                int(iterations), ctypes.byref(bad))
    if rc:
        raise OracleError(rc, f"oracle iterate_approx failed ({rc}), bad_row={bad.value}")
    out = dict(o)
    out["val"] = Rva[: o["nnz"]]
    out["bad_row"] = -1
    out["status"] = 0
    if B is None:
        out["n_uncovered"] = 0
    else:
        covered = np.zeros(n, bool)
        covered[o["col_idx"]] = True
        out["n_uncovered"] = int(((cfa == 0) & ~covered).sum())
    return out


def project_constraints(o, cf, B, rcond=1e-12):
    """R (an oracle result dict, built unconstrained) after imposing R^T B_c = B
    for the k columns of B (n x k): a new dict; also n_uncovered."""
    lib = _load()
    Bm = np.asarray(B, np.float64)
    Bm = np.ascontiguousarray(Bm if Bm.ndim == 2 else Bm.reshape(-1, 1))
    if Bm.shape[0] != len(cf):
        raise ValueError("B must be n x k")
    k = Bm.shape[1]
    va = np.array(o["val"], np.float64, copy=True)
    rp = np.ascontiguousarray(o["row_ptr"], np.int32)
    ci = np.ascontiguousarray(o["col_idx"], np.int32)
    cfa = np.ascontiguousarray(cf, np.int8)
    unc = ctypes.c_int64(0)
    rc = lib.orc_project_k(len(cfa), o["n_c"], _ptr(rp), _ptr(ci), _ptr(va), _ptr(cfa), _ptr(Bm), k, float(rcond),
                           ctypes.byref(unc))
    if rc:
        raise OracleError(rc, f"oracle project_k failed ({rc})")
    out = dict(o)
    out["val"] = va
    out["n_uncovered"] = unc.value
    return out
