"""Seeded synthetic inputs: upwind finite-difference advection-diffusion matrices.

This module only *generates inputs* (a CSR matrix A, a C/F marker and a
constraint vector B).  It holds none of the restriction-setup arithmetic, so
both the CPU oracle and the GPU path can draw their inputs from it.

The paper's own advection-diffusion tests (Section 4.2, constant and
recirculating flow) use upwind DG matrices from PyMFEM, which are not
available here; these finite-difference operators stand in for them.  They
keep the properties the method relies on: an upwinded, nonsymmetric,
diagonally dominant M-matrix whose character moves from advective to
diffusive as the diffusion constant grows.

Conventions
-----------
* Interior nodes only; Dirichlet values are eliminated (neighbours outside the
  grid are dropped).
* 0-based lexicographic numbering with x fastest:
  ``idx = ix + N*iy`` (2D) and ``idx = ix + N*(iy + N*iz)`` (3D).
* Grid spacing ``h = L/(N+1)``; node ``ix`` sits at ``x0 + (ix+1) h``.
* Diffusion ``-eps * Laplacian``:
  - 5-point: ``eps/h^2 * (4 | -1 x4)``;
  - compact 9-point: ``eps/(6 h^2) * (20 | -4 edges, -1 corners)``;
  - 7-point (3D): ``eps/h^2 * (6 | -1 x6)``.
* Advection ``b . grad u`` by first-order upwinding on the edge neighbours,
  with ``b`` evaluated at the node: for ``b_x > 0`` the west neighbour gets
  ``-b_x/h`` and the centre ``+b_x/h``; for ``b_x < 0`` the east neighbour gets
  ``-|b_x|/h`` and the centre ``+|b_x|/h`` (same per axis).  A zero component
  adds nothing.
* C-points: every index divisible by the coarsening factor ``k``.
* Columns are ascending within each row; no stored zeros; int32 indices and
  float64 values.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Problem:
    """One setup input: A (CSR), C/F marker, constraint vector B and degree ell."""

    name: str
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float64 [nnz]
    cf: np.ndarray  # int8 [n], 1 = C, 0 = F
    B: Optional[np.ndarray]  # float64 [n] or None (unconstrained)
    ell: int
    meta: dict = dataclasses.field(default_factory=dict)
    theta: float = 0.0  # strength threshold of the pattern (0: every stored nonzero)
    agg: Optional[np.ndarray] = None  # int32 [n]: root C-point of each point's aggregate, or -1

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))


# ----------------------------------------------------------------------------
# Stencil assembly
# ----------------------------------------------------------------------------

def _assemble(shape: Tuple[int, ...], offsets: List[Tuple[int, ...]], coef: List[np.ndarray]):
    """Assemble a CSR matrix from per-node stencil coefficients.

    ``offsets`` are neighbour offsets (d0, d1, ...) in grid coordinates with
    axis 0 fastest; ``coef[k]`` is an array over the grid giving the coefficient
    of offset k at every node.  Offsets are sorted by linear index so that the
    columns of every row come out ascending.
    """
    dims = len(shape)
    strides = [1]
    for d in range(1, dims):
        strides.append(strides[-1] * shape[d - 1])
    n = int(np.prod(shape))
    order = sorted(range(len(offsets)), key=lambda k: sum(o * s for o, s in zip(offsets[k], strides)))
    # grid coordinates, axis 0 fastest: reshape index as (..., axis1, axis0)
    grids = np.meshgrid(*[np.arange(s, dtype=np.int64) for s in reversed(shape)], indexing="ij")
    coords = [g.reshape(-1) for g in reversed(grids)]  # coords[d] for axis d, flattened lexicographically
    idx = np.arange(n, dtype=np.int64)
    cols = np.empty((n, len(offsets)), dtype=np.int64)
    vals = np.zeros((n, len(offsets)), dtype=np.float64)
    keep = np.zeros((n, len(offsets)), dtype=bool)
    for slot, k in enumerate(order):
        off = offsets[k]
        ok = np.ones(n, dtype=bool)
        lin = idx.copy()
        for d in range(dims):
            c = coords[d] + off[d]
            ok &= (c >= 0) & (c < shape[d])
            lin += off[d] * strides[d]
        v = np.asarray(coef[k], dtype=np.float64).reshape(-1)
        cols[:, slot] = lin
        vals[:, slot] = v
        keep[:, slot] = ok & (v != 0.0)
    counts = keep.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[keep].astype(np.int32)
    val = vals[keep]
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32")
    return n, row_ptr.astype(np.int32), col_idx, val


def _coords(shape, h, x0):
    """Node coordinates per axis (axis 0 fastest), each shaped like the flattened grid."""
    grids = np.meshgrid(*[x0 + (np.arange(s) + 1) * h for s in reversed(shape)], indexing="ij")
    return [g.reshape(-1) for g in reversed(grids)]


def _upwind(b_axis: np.ndarray, h: float):
    """First-order upwind coefficients on one axis: (centre, minus-neighbour, plus-neighbour)."""
    bp = np.maximum(b_axis, 0.0) / h
    bm = np.maximum(-b_axis, 0.0) / h
    return bp + bm, -bp, -bm


def advdiff_2d_5pt(N: int, eps: float, b: Callable | Tuple[float, float], *, domain=(0.0, 1.0)):
    """2D -eps*Lap u + b.grad u, 5-point diffusion + first-order upwind advection."""
    x0, x1 = domain
    h = (x1 - x0) / (N + 1)
    shape = (N, N)
    X, Y = _coords(shape, h, x0)
    if callable(b):
        bx, by = b(X, Y)
    else:
        bx = np.full(X.shape, float(b[0]))
        by = np.full(X.shape, float(b[1]))
    d = eps / (h * h)
    cxc, cxw, cxe = _upwind(np.asarray(bx, dtype=np.float64), h)
    cyc, cys, cyn = _upwind(np.asarray(by, dtype=np.float64), h)
    offsets = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    coef = [4 * d + cxc + cyc, -d + cxw, -d + cxe, -d + cys, -d + cyn]
    return _assemble(shape, offsets, coef)


def advdiff_2d_9pt(N: int, eps: float, b: Callable | Tuple[float, float], *, domain=(0.0, 1.0)):
    """2D compact 9-point diffusion eps/(6h^2)*(20|-4|-1) + upwind advection on edge neighbours."""
    x0, x1 = domain
    h = (x1 - x0) / (N + 1)
    shape = (N, N)
    X, Y = _coords(shape, h, x0)
    if callable(b):
        bx, by = b(X, Y)
    else:
        bx = np.full(X.shape, float(b[0]))
        by = np.full(X.shape, float(b[1]))
    d = eps / (6.0 * h * h)
    cxc, cxw, cxe = _upwind(np.asarray(bx, dtype=np.float64), h)
    cyc, cys, cyn = _upwind(np.asarray(by, dtype=np.float64), h)
    offsets = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1), (-1, -1), (1, -1), (-1, 1), (1, 1)]
    corner = np.full(X.shape, -d)
    coef = [20 * d + cxc + cyc, -4 * d + cxw, -4 * d + cxe, -4 * d + cys, -4 * d + cyn,
            corner, corner, corner, corner]
    return _assemble(shape, offsets, coef)


def advdiff_3d_7pt(N: int, eps: float, b: Tuple[float, float, float]):
    """3D 7-point diffusion + first-order upwind advection on [0,1]^3."""
    h = 1.0 / (N + 1)
    shape = (N, N, N)
    n = N ** 3
    d = eps / (h * h)
    cc = np.full(n, 6 * d)
    minus, plus = [], []
    for ax in range(3):
        c0, cm, cp = _upwind(np.full(n, float(b[ax])), h)
        cc = cc + c0
        minus.append(-d + cm)
        plus.append(-d + cp)
    offsets = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    coef = [cc, minus[0], plus[0], minus[1], plus[1], minus[2], plus[2]]
    return _assemble(shape, offsets, coef)


def cf_every_k(shape: Sequence[int], k: int) -> np.ndarray:
    """C/F marker: node is a C-point iff every grid index is divisible by k (axis 0 fastest)."""
    grids = np.meshgrid(*[np.arange(s) for s in reversed(shape)], indexing="ij")
    c = np.ones(grids[0].shape, dtype=bool)
    for g in grids:
        c &= (g % k) == 0
    return c.reshape(-1).astype(np.int8)


def _problem(name, mat, shape, k, ell, B="ones", meta=None):
    n, rp, ci, va = mat
    cf = cf_every_k(shape, k)
    if isinstance(B, str) and B == "ones":
        Bv = np.ones(n, dtype=np.float64)
    else:
        Bv = B
    return Problem(name, n, rp, ci, va, cf, Bv, ell, dict(meta or {}, shape=tuple(shape), k=k))


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------

B_CONST = (math.cos(math.pi / 6), math.sin(math.pi / 6))


def cfg1(B="ones") -> Problem:
    """32x32 interior grid, 5-point upwind, eps=0.1, b=(cos pi/6, sin pi/6), C=(even,even), ell=1."""
    return _problem("cfg1_32x32_5pt_l1", advdiff_2d_5pt(32, 0.1, B_CONST), (32, 32), 2, 1, B,
                    dict(eps=0.1))


def cfg2(eps_list=(1e-6, 1e-2, 1.0), N=512, B="ones") -> List[Problem]:
    """512x512 5-point upwind, one matrix per eps in {1e-6, 1e-2, 1}, C every 2nd node, ell=2."""
    return [_problem(f"cfg2_{N}x{N}_5pt_eps{e:g}_l2", advdiff_2d_5pt(N, e, B_CONST), (N, N), 2, 2, B,
                     dict(eps=e)) for e in eps_list]


def recirc_b(X, Y):
    """Recirculating flow b(x,y) = (y(1-x^2), -x(1-y^2)) on [-1,1]^2."""
    return Y * (1.0 - X * X), -X * (1.0 - Y * Y)


def cfg3(N=2048, ell=2, B="ones") -> Problem:
    """Recirculating flow on [-1,1]^2, 9-point upwind, eps=1e-4, C every 3rd node, ell=2."""
    return _problem(f"cfg3_{N}x{N}_9pt_recirc_l{ell}", advdiff_2d_9pt(N, 1e-4, recirc_b, domain=(-1.0, 1.0)),
                    (N, N), 3, ell, B, dict(eps=1e-4))


def cfg4(nmat=64, seed=0, side_range=(64, 768), B="ones") -> List[Problem]:
    """Batched set: nmat 5-point upwind matrices, side ~ U{64..768}, eps = 10^U(-6,0),
    flow angle ~ U[0, 2pi), ell ~ U{1,2}, C every 2nd node.

    Draws from ``numpy.random.default_rng(seed)`` per matrix in the order
    side, log10(eps), angle, ell.
    """
    rng = np.random.default_rng(seed)
    out = []
    for m in range(nmat):
        side = int(rng.integers(side_range[0], side_range[1] + 1))
        eps = float(10.0 ** rng.uniform(-6.0, 0.0))
        ang = float(rng.uniform(0.0, 2.0 * math.pi))
        ell = int(rng.integers(1, 3))
        b = (math.cos(ang), math.sin(ang))
        out.append(_problem(f"cfg4_m{m}_{side}x{side}_l{ell}", advdiff_2d_5pt(side, eps, b), (side, side), 2, ell, B,
                            dict(eps=eps, angle=ang)))
    return out


def cfg5(N=128, ell=2, B="ones") -> Problem:
    """3D 7-point upwind on 128^3, eps=1e-3, b=(1,0.5,0.25)/|b|, C every 2nd node, ell=2."""
    bb = np.array([1.0, 0.5, 0.25])
    bb = bb / np.linalg.norm(bb)
    return _problem(f"cfg5_{N}^3_7pt_l{ell}", advdiff_3d_7pt(N, 1e-3, tuple(bb)), (N, N, N), 2, ell, B,
                    dict(eps=1e-3))


# ----------------------------------------------------------------------------
# Small randomised cases for tests
# ----------------------------------------------------------------------------

def small_2d(N: int, *, stencil: int = 5, eps: float = 0.1, angle: float = math.pi / 6, k: int = 2,
             ell: int = 1, B="ones") -> Problem:
    b = (math.cos(angle), math.sin(angle))
    if stencil == 5:
        mat = advdiff_2d_5pt(N, eps, b)
    elif stencil == 9:
        mat = advdiff_2d_9pt(N, eps, b)
    else:
        raise ValueError(stencil)
    return _problem(f"small{stencil}_{N}_l{ell}", mat, (N, N), k, ell, B, dict(eps=eps, angle=angle))


def small_3d(N: int, *, eps: float = 0.1, b=(1.0, 0.5, 0.25), k: int = 2, ell: int = 1, B="ones") -> Problem:
    return _problem(f"small3d_{N}_l{ell}", advdiff_3d_7pt(N, eps, b), (N, N, N), k, ell, B, dict(eps=eps))


def random_sparse(n: int, density: float, seed: int, *, c_frac: float = 0.3, ell: int = 2,
                  nonsym_pattern: bool = True, dominant: bool = True, B="random") -> Problem:
    """A random sparse matrix with a (possibly structurally nonsymmetric) pattern.

    Diagonal entries are set so the matrix is strictly diagonally dominant when
    ``dominant`` is true; otherwise the diagonal is random (pivoting needed).
    """
    rng = np.random.default_rng(seed)
    M = (rng.random((n, n)) < density)
    if not nonsym_pattern:
        M = M | M.T
    np.fill_diagonal(M, False)
    vals = np.where(M, -rng.uniform(0.1, 1.0, (n, n)), 0.0)
    if dominant:
        diag = np.abs(vals).sum(axis=1) + rng.uniform(0.5, 1.5, n)
    else:
        diag = rng.uniform(-1.0, 1.0, n)
        vals = vals * rng.choice([-1.0, 1.0], (n, n))
    vals[np.arange(n), np.arange(n)] = diag
    rp = [0]
    ci, va = [], []
    for r in range(n):
        cols = np.nonzero(vals[r])[0]
        ci.extend(cols.tolist())
        va.extend(vals[r, cols].tolist())
        rp.append(len(ci))
    cf = (rng.random(n) < c_frac).astype(np.int8)
    if B == "random":
        Bv = rng.uniform(0.5, 1.5, n)
    elif B == "ones":
        Bv = np.ones(n)
    else:
        Bv = B
    return Problem(f"rand_n{n}_s{seed}", n, np.asarray(rp, np.int32), np.asarray(ci, np.int32),
                   np.asarray(va, np.float64), cf, Bv, ell, dict(seed=seed))


def greedy_aggregates(p: Problem) -> Problem:
    """The same matrix with an aggregation-based C/F splitting: a sequential
    greedy aggregation of A's graph (a point whose neighbours are all still
    free seeds an aggregate with them; free points left join the aggregate of
    their first aggregated neighbour, or seed a singleton).  Seeds become the
    C-points, every other point an F-point; agg[j] = the seed of j's
    aggregate.  The splitting is an input of the setup, like cf."""
    n = p.n
    rp, ci = p.row_ptr, p.col_idx
    agg = np.full(n, -1, np.int64)
    for i in range(n):
        nb = ci[rp[i]:rp[i + 1]]
        nb = nb[nb != i]
        if agg[i] < 0 and np.all(agg[nb] < 0):
            agg[i] = i
            agg[nb] = i
    for i in range(n):
        if agg[i] < 0:
            nb = ci[rp[i]:rp[i + 1]]
            nb = nb[(nb != i) & (agg[nb] >= 0)]
            agg[i] = agg[nb[0]] if len(nb) else i
    cf = (agg == np.arange(n)).astype(np.int8)
    return dataclasses.replace(p, name=p.name + "_agg", cf=cf, agg=agg.astype(np.int32))
